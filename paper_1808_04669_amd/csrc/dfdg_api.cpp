// C ABI of the library (declared in include/dfdg.h): context management, workspace
// layout, and the host-side orchestration of the hot path (residual -> condensation ->
// facet PCG -> recovery, inside TVD-RK3).  Kernels are enqueued on the context stream;
// the host only reads back PCG scalars every few iterations.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "dfdg.h"
#include "dfdg_amg.h"
#include "dfdg_kernels.h"
#include "dfdg_setup.h"

using namespace dfdg;

struct dfdg_mesh {
  MeshHost m;
};

constexpr int kHistSlots = 7;

constexpr int kHintRuns = 3;  // PCG runs whose iteration counts size the first chunk

struct dfdg_ctx {
  dfdg_params prm{};
  hipStream_t stream = nullptr;
  HostSetup hs;
  int dim = 2;  // 2: triangles, 3: tetrahedra
  int K = 0, P = 0, NF = 0, T = 0, E = 0;
  long nU = 0, nL = 0;
  size_t ws_need = 0;
  char* ws = nullptr;
  bool bound = false;
  DevGeo g{};
  DevTabs tb{};
  DevBsr A{};
  // work buffers
  double *Lbuf = nullptr, *q = nullptr, *gv = nullptr, *lamw = nullptr, *r = nullptr, *rb = nullptr, *z = nullptr,
         *p[2] = {nullptr, nullptr}, *Sp = nullptr, *Ustage = nullptr, *hist[kHistSlots][kHistDepth] = {}, *evaltab = nullptr,
         *partials = nullptr, *diagres = nullptr, *r64 = nullptr, *xpart = nullptr;
  // warm starts of the forward stages formed ahead: while the host waits for the end of
  // one stage's solve, the GPU forms the next stage's start value (it depends only on that
  // stage's history) into gbuf
  double* gbuf[3] = {nullptr, nullptr, nullptr};
  bool gready[3] = {false, false, false};
  int defer_slot = -1;
  hipEvent_t sc_event = nullptr;
  float *L32 = nullptr, *x32 = nullptr, *r32 = nullptr, *r32b = nullptr, *z32 = nullptr, *p32[2] = {nullptr, nullptr},
        *Sp32 = nullptr;
  PcgBufs pb{}, pb32{}, pbt{};  // FP64 PCG / refinement, FP32 inner PCG, kernel timing
  // adjoint buffers
  double *Ustages[3] = {nullptr, nullptr, nullptr}, *Ybar = nullptr, *Wbuf = nullptr;
  // multiplier history per slot: 0-2 the forward stages (TVD-RK3; the first three of RK4, the
  // single one of forward Euler), 3-5 the adjoint stage solves, 6 RK4's fourth stage
  int hist_count[kHistSlots] = {};
  // the forward integrator whose stage solves the history 0-2, 6 holds (0 none, 1 TVD-RK3,
  // 2 RK4, 3 forward Euler): another one starts from an empty history
  int integrator = 0;
  // multigrid preconditioner
  AmgHierarchy H;
  MgDev mg;
  // PCG iterations captured as HIP graphs (kernel arguments fixed: the solve runs in lamx)
  double* lamx = nullptr;
  hipStream_t cap_stream = nullptr;
  // one graph per iteration parity ([1]: odd iterations, [0]: even), FP64 and FP32 PCG
  // captured PCG iterations: [2j + p] holds 2^j consecutive iterations (j = 0, 1, 2)
  // starting with parity p (0 even, 1 odd)
  hipGraphExec_t graph64[6] = {}, graph32[6] = {};
  // start values of the forward stage solves projected onto earlier solutions
  // (DFDG_EXTRAPOLATE_PROJECT): basis X (images SX, S-norms squared pjnrm) of proj_nb
  // vectors, and a ring of the latest proj_raw solutions and right-hand sides (next slot
  // proj_head) that the basis is rebuilt from when full
  bool proj_on = false, proj_req = false;
  int proj_nb = 0, proj_raw = 0, proj_head = 0;
  double *pjX[kProjMax] = {}, *pjSX[kProjMax] = {}, *pjRawL[kProjKeep] = {}, *pjRawG[kProjKeep] = {};
  double *pjx0 = nullptr, *pjnrm = nullptr, *pjT = nullptr, *pjcA = nullptr, *pjcB = nullptr, *pjpart = nullptr;
  // iterations of the last kHintRuns runs, newest first (FP64 solve / FP32 inner solve)
  int iters_hint[2][kHintRuns] = {};
  PcgScalars* pinned = nullptr;
  double* noalloc = nullptr;  // device address of the static scratch of dfdg_diagnostics_noalloc
  std::string err;
};

// Start values formed ahead are void once a history changes other than by a solve.
static void invalidate_guesses(dfdg_ctx* ctx) {
  for (int i = 0; i < 3; ++i) ctx->gready[i] = false;
  ctx->defer_slot = -1;
  // the projection basis holds the same history
  ctx->proj_nb = ctx->proj_raw = ctx->proj_head = 0;
}

static thread_local std::string g_mesh_err;

static int fail(dfdg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPC(x)                                                                           \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) return fail(ctx, DFDG_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define NEED_BOUND(ctx)                                                                   \
  do {                                                                                    \
    if (!(ctx)) return DFDG_E_INVALID_ARG;                                                \
    if (!(ctx)->bound) return fail(ctx, DFDG_E_WORKSPACE, "no workspace bound");          \
  } while (0)

// Element steps on triangles or tetrahedra (the facet kernels are shared).
static hipError_t el_residual(dfdg_ctx* ctx, bool f32, const double* U, void* L, hipStream_t s) {
  if (ctx->dim == 3) return launch_residual3(ctx->K, ctx->g, ctx->tb, U, (double*)L, ctx->prm.nu, s);
  return launch_residual(ctx->K, f32, ctx->g, ctx->tb, U, L, ctx->prm.nu, s);
}
static hipError_t el_cond_rhs(dfdg_ctx* ctx, bool f32, const void* F, hipStream_t s) {
  if (ctx->dim == 3) return launch_cond_rhs3(ctx->K, ctx->g, ctx->tb, (const double*)F, ctx->q, s);
  return launch_cond_rhs(ctx->K, f32, ctx->g, ctx->tb, F, ctx->q, s);
}
static hipError_t el_recover(dfdg_ctx* ctx, bool f32, const void* F, const double* lam, double* out, int mode,
                             double a, const double* Un, double b, const double* Us, double dt, hipStream_t s) {
  if (ctx->dim == 3) return launch_recover3(ctx->K, ctx->g, ctx->tb, (const double*)F, lam, out, mode, a, Un, b, Us, dt, s);
  return launch_recover(ctx->K, f32, ctx->g, ctx->tb, F, lam, out, mode, a, Un, b, Us, dt, s);
}
static hipError_t el_load_vector(dfdg_ctx* ctx, const double* fq, double* F, hipStream_t s) {
  if (ctx->dim == 3) return launch_load_vector3(ctx->K, ctx->hs.tabs.nqp, ctx->g, ctx->tb, fq, F, s);
  return launch_load_vector(ctx->K, ctx->hs.tabs.nqp, ctx->g, ctx->tb, fq, F, s);
}
static hipError_t el_diagnostics(dfdg_ctx* ctx, const double* U, double* part, double* res, hipStream_t s) {
  if (ctx->dim == 3) return launch_diagnostics3(ctx->K, ctx->g, ctx->tb, U, part, res, s);
  return launch_diagnostics(ctx->K, ctx->g, ctx->tb, U, part, res, s);
}

// ---------------------------------------------------------------------------------------
// mesh
// ---------------------------------------------------------------------------------------
extern "C" int dfdg_mesh_create(int dim, int n_elem, const double* xyz, const double* period, dfdg_mesh** out) {
  if (!out) { g_mesh_err = "out is NULL"; return DFDG_E_INVALID_ARG; }
  *out = nullptr;
  if (dim != 2 && dim != 3) { g_mesh_err = "dim must be 2 or 3"; return DFDG_E_INVALID_ARG; }
  if (n_elem < 2 || !xyz || !period) { g_mesh_err = "need >= 2 elements, coordinates and a period"; return DFDG_E_INVALID_ARG; }
  // a period component 0 gives that direction walls (boundary facets, no flow)
  for (int d = 0; d < dim; ++d)
    if (!std::isfinite(period[d]) || period[d] < 0) {
      g_mesh_err = "period must be finite and >= 0";
      return DFDG_E_INVALID_ARG;
    }
  const long nco = (long)dim * (dim + 1) * n_elem;
  for (long i = 0; i < nco; ++i)
    if (!std::isfinite(xyz[i])) { g_mesh_err = "non-finite vertex coordinate"; return DFDG_E_INVALID_ARG; }
  auto* m = new dfdg_mesh;
  std::string err;
  int rc = dim == 3 ? build_mesh3(n_elem, xyz, period, m->m, err) : build_mesh(n_elem, xyz, period, m->m, err);
  if (rc) { g_mesh_err = err; delete m; return DFDG_E_MESH; }
  *out = m;
  return DFDG_OK;
}
extern "C" void dfdg_mesh_destroy(dfdg_mesh* m) { delete m; }
extern "C" const char* dfdg_mesh_last_error(void) { return g_mesh_err.c_str(); }
extern "C" int dfdg_mesh_counts(const dfdg_mesh* m, int* T, int* E) {
  if (!m || !T || !E) return DFDG_E_INVALID_ARG;
  *T = m->m.T;
  *E = m->m.E;
  return DFDG_OK;
}
extern "C" int dfdg_mesh_facets(const dfdg_mesh* m, int32_t* f) {
  if (!m || !f) return DFDG_E_INVALID_ARG;
  for (int F = 0; F < m->m.E; ++F) {
    f[4 * F + 0] = m->m.fL[F];
    f[4 * F + 1] = m->m.fLloc[F];
    f[4 * F + 2] = m->m.fR[F];
    f[4 * F + 3] = m->m.fRloc[F];
  }
  return DFDG_OK;
}

extern "C" int dfdg_mesh_set_outflow(dfdg_mesh* m, const int32_t* open) {
  if (!m || !open) {
    g_mesh_err = "null pointer";
    return DFDG_E_INVALID_ARG;
  }
  std::vector<uint8_t> f(m->m.E, 0);
  for (int F = 0; F < m->m.E; ++F) {
    if (open[F] != 0 && open[F] != 1) {
      g_mesh_err = "outflow marks must be 0 or 1";
      return DFDG_E_INVALID_ARG;
    }
    if (open[F] && m->m.fR[F] >= 0) {
      g_mesh_err = "facet " + std::to_string(F) + " is not a boundary facet";
      return DFDG_E_INVALID_ARG;
    }
    f[F] = (uint8_t)open[F];
  }
  m->m.fopen = std::move(f);
  return DFDG_OK;
}

// ---------------------------------------------------------------------------------------
// context and workspace
// ---------------------------------------------------------------------------------------
extern "C" void dfdg_params_default(dfdg_params* p) {
  if (!p) return;
  p->k = 2;
  p->nu = 0.0;
  p->alpha = 2.0;
  p->precision = DFDG_FP64;
  p->cg_rtol = 1e-12;
  p->cg_maxit = 20000;
  p->precond = DFDG_JACOBI;
  p->ir_rtol = 1e-10;
  p->inner_rtol = 1e-4;
  p->extrapolate = 0;
  p->graphs = 1;
  p->mg_fp32 = 1;
  p->mg_fine_fp16 = 1;
  p->facet_blocks = 0;
  p->matrix_free = 0;
  p->mixed_solver = 1;
  p->local_space = DFDG_LOCAL_FE3;
  p->mg_fine_smooth = 2;
}

static_assert(DFDG_HISTORY_DEPTH == kHistDepth, "history depth of the ABI and the kernels");
static_assert(DFDG_EXTRAPOLATE_ADAPTIVE == kExtrapAdaptive, "adaptive extrapolation value");

static int check_params(const dfdg_params* p, std::string& e) {
  if (p->k < 1 || p->k > kMaxK) { e = "k must be in 1..3"; return -1; }
  if (!(p->nu >= 0) || !std::isfinite(p->nu)) { e = "nu must be finite and >= 0"; return -1; }
  if (!(p->alpha > 0) || !std::isfinite(p->alpha)) { e = "alpha must be finite and > 0"; return -1; }
  if (p->precision != DFDG_FP64 && p->precision != DFDG_MIXED) { e = "precision must be DFDG_FP64 or DFDG_MIXED"; return -1; }
  if (!(p->cg_rtol > 0 && p->cg_rtol < 1)) { e = "cg_rtol must be in (0,1)"; return -1; }
  if (p->cg_maxit < 1) { e = "cg_maxit must be >= 1"; return -1; }
  if (p->precond != DFDG_JACOBI && p->precond != DFDG_BLOCK_JACOBI && p->precond != DFDG_AMG) {
    e = "unknown preconditioner";
    return -1;
  }
  if (p->precision == DFDG_MIXED) {
    if (!(p->ir_rtol > 0 && p->ir_rtol < 1)) { e = "ir_rtol must be in (0,1)"; return -1; }
    if (!(p->inner_rtol > 0 && p->inner_rtol < 1)) { e = "inner_rtol must be in (0,1)"; return -1; }
  }
  if (p->extrapolate < 0 || p->extrapolate > DFDG_EXTRAPOLATE_PROJECT) {
    e = "extrapolate must be in 0..4, DFDG_EXTRAPOLATE_ADAPTIVE or DFDG_EXTRAPOLATE_PROJECT";
    return -1;
  }
  if (p->extrapolate == DFDG_EXTRAPOLATE_PROJECT && p->precision != DFDG_FP64) {
    e = "DFDG_EXTRAPOLATE_PROJECT needs an FP64 context";
    return -1;
  }
  if (p->graphs != 0 && p->graphs != 1) { e = "graphs must be 0 or 1"; return -1; }
  if (p->mg_fp32 != 0 && p->mg_fp32 != 1) { e = "mg_fp32 must be 0 or 1"; return -1; }
  if (p->mg_fine_fp16 != 0 && p->mg_fine_fp16 != 1) { e = "mg_fine_fp16 must be 0 or 1"; return -1; }
  if (p->facet_blocks < 0 || p->facet_blocks > 1024) { e = "facet_blocks must be in 0..1024"; return -1; }
  if (p->matrix_free != 0 && p->matrix_free != 1) { e = "matrix_free must be 0 or 1"; return -1; }
  if (p->mixed_solver != 0 && p->mixed_solver != 1) { e = "mixed_solver must be 0 or 1"; return -1; }
  if (p->mg_fine_smooth < 1 || p->mg_fine_smooth > 3) { e = "mg_fine_smooth must be in 1..3"; return -1; }
  if (p->local_space != DFDG_LOCAL_FE3 && p->local_space != DFDG_LOCAL_FE4) {
    e = "local_space must be DFDG_LOCAL_FE3 or DFDG_LOCAL_FE4";
    return -1;
  }
  return 0;
}

extern "C" int dfdg_ctx_create(const dfdg_mesh* mesh, const dfdg_params* prm, void* stream, dfdg_ctx** out) {
  if (!out) return DFDG_E_INVALID_ARG;
  *out = nullptr;
  if (!mesh || !prm) return DFDG_E_INVALID_ARG;
  auto* ctx = new dfdg_ctx;
  ctx->prm = *prm;
  ctx->stream = (hipStream_t)stream;
  ctx->dim = mesh->m.dim;
  std::string e;
  if (check_params(prm, e)) {
    g_mesh_err = e;
    delete ctx;
    return DFDG_E_INVALID_ARG;
  }
  if (ctx->dim == 3) {  // what the tetrahedral path implements
    const char* why = prm->k > kMaxK3 ? "tetrahedral meshes: k must be 1 or 2"
                      : prm->precision != DFDG_FP64 ? "tetrahedral meshes: FP64 only"
                      : prm->local_space != DFDG_LOCAL_FE3 ? "tetrahedral meshes: local_space must be DFDG_LOCAL_FE3"
                                                           : nullptr;
    if (why) {
      g_mesh_err = why;
      delete ctx;
      return DFDG_E_UNSUPPORTED;
    }
  } else if (prm->matrix_free) {
    g_mesh_err = "matrix_free: tetrahedral meshes only";
    delete ctx;
    return DFDG_E_UNSUPPORTED;
  }
  ctx->hs.fe4 = ctx->dim == 2 && prm->local_space == DFDG_LOCAL_FE4;
  if ((ctx->dim == 3 ? build_setup3(mesh->m, prm->k, prm->alpha, ctx->hs, e)
                     : build_setup(mesh->m, prm->k, prm->alpha, ctx->hs, e))) {
    g_mesh_err = e;
    delete ctx;
    return DFDG_E_MESH;
  }
  if (prm->precond == DFDG_AMG) {
    const HostSetup& h = ctx->hs;
    const int NFk = ctx->dim == 3 ? nF3(prm->k) : nF(prm->k);
    std::vector<double> z((size_t)h.E * NFk, 0.0);
    for (int F = 0; F < h.E; ++F) z[(size_t)F * NFk] = h.nearnull.empty() ? h.zdef[F] : h.nearnull[F];
    if (build_amg(h.E, NFk, (int)(h.cols.size() / h.E), h.cols, h.vals, z, h.singular, 0.08, 1000,
                  prm->mg_fine_smooth, ctx->H, e)) {
      g_mesh_err = e;
      delete ctx;
      return DFDG_E_MESH;
    }
    if ((int)ctx->H.lv.size() > kMaxLev) {
      g_mesh_err = "multigrid: too many levels";
      delete ctx;
      return DFDG_E_UNSUPPORTED;
    }
  }
  ctx->K = prm->k;
  ctx->P = ctx->dim == 3 ? nP3(ctx->K) : nP(ctx->K);
  ctx->NF = ctx->dim == 3 ? nF3(ctx->K) : nF(ctx->K);
  ctx->T = mesh->m.T;
  ctx->E = mesh->m.E;
  ctx->nU = (long)ctx->dim * ctx->P * ctx->T;
  ctx->nL = (long)ctx->NF * ctx->E;
  *out = ctx;
  return DFDG_OK;
}

extern "C" int dfdg_ctx_set_stream(dfdg_ctx* ctx, void* stream) {
  if (!ctx) return DFDG_E_INVALID_ARG;
  // work still queued on the previous stream (a recovery, a start value formed ahead)
  // finishes before any work on the new one
  if (ctx->bound && (hipStream_t)stream != ctx->stream) HIPC(hipStreamSynchronize(ctx->stream));
  ctx->stream = (hipStream_t)stream;
  return DFDG_OK;
}

extern "C" int dfdg_ctx_sizes(const dfdg_ctx* ctx, dfdg_sizes* s) {
  if (!ctx || !s) return DFDG_E_INVALID_ARG;
  s->T = ctx->T;
  s->E = ctx->E;
  s->k = ctx->K;
  s->P = ctx->P;
  s->n_f = ctx->NF;
  s->n_p = ctx->dim == 3 ? nPp3(ctx->K) : nPp(ctx->K);
  s->n_broken = ctx->nU;
  s->n_lambda = ctx->nL;
  s->n_bdm = (long)ctx->E * ctx->NF + (long)ctx->T * (ctx->dim * ctx->P - (ctx->dim + 1) * ctx->NF);
  s->nq_proj = ctx->hs.tabs.nqp;
  s->dim = ctx->dim;
  return DFDG_OK;
}

// Workspace carving: a first pass with base == nullptr only counts bytes.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

static int d3slots(const dfdg_ctx* ctx) { return ctx->dim == 3 ? kSlots3 : kSlots; }

static void carve(dfdg_ctx* ctx, char* base) {
  Carver c{base};
  const HostSetup& h = ctx->hs;
  const long T = ctx->T, E = ctx->E, NF = ctx->NF, nU = ctx->nU, nL = ctx->nL;
  const RefTables& tb = h.tabs;
  DevGeo& g = ctx->g;
  g.T = (int)T;
  g.E = (int)E;
  // one thread per facet row, or two for split rows (facet_split)
  g.fgrid = facet_grid_size((int)(E * facet_split((int)NF, d3slots(ctx))), ctx->prm.facet_blocks);
  const long dm = ctx->dim, nfac = dm + 1;
  g.Jinv = c.take<double>(dm * dm * T);
  g.detJ = c.take<double>(T);
  g.isq = c.take<double>(T);
  g.nbr = c.take<int>(nfac * T);
  g.code = c.take<int>(nfac * T);
  g.efacet = c.take<int>(nfac * T);
  g.nx = c.take<double>(nfac * T);
  g.ny = c.take<double>(nfac * T);
  g.nz = dm == 3 ? c.take<double>(nfac * T) : nullptr;
  g.flen = c.take<double>(nfac * T);
  g.sig = c.take<double>(nfac * T);
  g.sF = c.take<double>(nfac * T);
  g.G = c.take<double>(h.G.size());
  g.G4 = h.G4.empty() ? nullptr : c.take<double>(h.G4.size());
  g.qL = c.take<int>(E);
  g.qR = c.take<int>(E);
  g.zdef = c.take<double>(E);
  DevTabs& d = ctx->tb;
  d.Vv = c.take<double>(tb.Vv.size());
  d.Gv = c.take<double>(tb.Gv.size());
  d.Wv = c.take<double>(tb.vw.size());
  d.Vf = c.take<double>(tb.Vf.size());
  d.Gf = c.take<double>(tb.Gf.size());
  d.Wf = c.take<double>(tb.fw.size());
  d.Vp = c.take<double>(tb.Vp.size());
  d.Wp = c.take<double>(tb.pw.size());
  d.Dh = c.take<double>(tb.Dh.size());
  d.Ch = c.take<double>(tb.Ch.size());
  d.Zh = tb.Zh.empty() ? nullptr : c.take<double>(tb.Zh.size());
  d.fpidx = tb.fpidx.empty() ? nullptr : c.take<int>(tb.fpidx.size());
  d.Qf = tb.Qf.empty() ? nullptr : c.take<double>(tb.Qf.size());
  DevBsr& A = ctx->A;
  A.ns = d3slots(ctx);
  A.cols = c.take<int>(h.cols.size());
  A.vals = c.take<double>(h.vals.size());
  A.dinv = c.take<double>(h.dinv.size());
  A.binv = c.take<double>(h.binv.size());
  const bool mixed = ctx->prm.precision == DFDG_MIXED;
  // FP32 copies of S (and of the multigrid data) for the mixed form or an FP32 V-cycle
  const bool f32 = mixed || (ctx->prm.precond == DFDG_AMG && ctx->prm.mg_fp32);
  A.vals32 = f32 ? c.take<float>(h.vals.size()) : nullptr;
  A.dinv32 = f32 ? c.take<float>(h.dinv.size()) : nullptr;
  A.binv32 = f32 ? c.take<float>(h.binv.size()) : nullptr;
  const bool f16 = ctx->prm.precond == DFDG_AMG && (mixed || ctx->prm.mg_fp32) && ctx->prm.mg_fine_fp16;
  A.vals16 = f16 ? c.take<uint32_t>((size_t)nPairs(NF, A.ns) * E) : nullptr;
  const bool amg = ctx->prm.precond == DFDG_AMG;
  A.tdef = amg ? c.take<double>(nL) : nullptr;
  A.tdef32 = amg && f32 ? c.take<float>(nL) : nullptr;
  // work
  ctx->Lbuf = c.take<double>(nU);
  ctx->q = c.take<double>(nfac * NF * T);
  // the matrix-free products use q for the face contributions: the condensation right-hand
  // side in it has been gathered into g before the PCG runs, and nothing reads it after
  A.mfq = ctx->prm.matrix_free ? ctx->q : nullptr;
  A.mfCh = d.Ch;
  A.mfDh = d.Dh;
  A.mfQf = d.Qf;
  A.mfK = ctx->K;
  ctx->gv = c.take<double>(nL);
  ctx->lamw = c.take<double>(nL);
  ctx->lamx = c.take<double>(nL);
  ctx->r = c.take<double>(nL);
  ctx->rb = c.take<double>(nL);  // second residual buffer (multigrid PCG alternates)
  ctx->z = c.take<double>(nL);
  ctx->p[0] = c.take<double>(nL);
  ctx->p[1] = c.take<double>(nL);
  ctx->Sp = c.take<double>(nL);
  ctx->Ustage = c.take<double>(nU);
  for (int s = 0; s < kHistSlots; ++s)
    for (int j = 0; j < kHistDepth; ++j) ctx->hist[s][j] = c.take<double>(nL);
  for (int s = 0; s < 3; ++s) ctx->gbuf[s] = c.take<double>(nL);
  ctx->proj_on = ctx->prm.extrapolate == DFDG_EXTRAPOLATE_PROJECT;
  if (ctx->proj_on) {
    for (int i = 0; i < kProjMax; ++i) {
      ctx->pjX[i] = c.take<double>(nL);
      ctx->pjSX[i] = c.take<double>(nL);
    }
    for (int i = 0; i < kProjKeep; ++i) {
      ctx->pjRawL[i] = c.take<double>(nL);
      ctx->pjRawG[i] = c.take<double>(nL);
    }
    ctx->pjx0 = c.take<double>(nL);
    ctx->pjnrm = c.take<double>(kProjMax);
    ctx->pjT = c.take<double>((size_t)kProjMax * kProjMax);
    ctx->pjcA = c.take<double>(kProjMax);
    ctx->pjcB = c.take<double>(kProjMax);
    ctx->pjpart = c.take<double>((size_t)kProjGrid * kProjPart);
  }
  ctx->evaltab = c.take<double>((size_t)kMaxEvalPts * ctx->P);
  const long maxblk = std::max((T + 127) / 128, (E + 255) / 256) + 1;
  ctx->partials = c.take<double>(4 * maxblk);
  ctx->diagres = c.take<double>(4);
  ctx->xpart = c.take<double>(kExtrapParts);
  const long G = g.fgrid;
  for (PcgBufs* pb : {&ctx->pb, &ctx->pb32, &ctx->pbt}) {
    pb->sc = c.take<PcgScalars>(1);
    pb->gg = c.take<double>(3 * G);
    pb->rz[0] = c.take<double>(2 * G);
    pb->rz[1] = c.take<double>(2 * G);
    pb->pq = c.take<double>(2 * G);
  }
  if (mixed) {
    ctx->L32 = c.take<float>(nU);
    ctx->x32 = c.take<float>(nL);
    ctx->r32 = c.take<float>(nL);
    ctx->r32b = c.take<float>(nL);
    ctx->z32 = c.take<float>(nL);
    ctx->p32[0] = c.take<float>(nL);
    ctx->p32[1] = c.take<float>(nL);
    ctx->Sp32 = c.take<float>(nL);
    ctx->r64 = c.take<double>(nL);
  }
  for (int s = 0; s < 3; ++s) ctx->Ustages[s] = c.take<double>(nU);
  ctx->Ybar = c.take<double>(nU);
  ctx->Wbuf = c.take<double>(nU);
  // multigrid hierarchy: operators of levels >= 1, transfer operators, level vectors
  MgDev& mg = ctx->mg;
  mg = MgDev{};
  const AmgHierarchy& H = ctx->H;
  mg.nlev = (int)H.lv.size();
  // lanes per row: the largest power of two not above the mean row length / div (<= 64)
  // returns whether the rows were packed (decided from the matrix, never from a pointer:
  // the sizing pass carves with a null base)
  auto take_csr = [&](const Csr& M, DevCsr& D, int div, bool pack = false, bool half = false) -> bool {
    D.n = M.n;
    const double avg = M.n ? (double)M.nnz() / M.n : 1.0;
    D.lpr = 1;
    while (D.lpr < 64 && 2 * D.lpr * div <= avg) D.lpr *= 2;
    int wmax = 1;
    for (int i = 0; i < M.n; ++i) wmax = std::max(wmax, M.ptr[i + 1] - M.ptr[i]);
    // short rows: one lane reads its whole row at once (16-byte loads; rows of up to 16
    // entries when they are packed into FP16 with 16-bit columns, 4 entries per load)
    const bool pack16 = pack && wmax <= 16 && M.m < 65536;
    if (wmax <= 4 || pack16) D.lpr = 1;
    D.w = wmax <= 4 ? 4 : pack16 ? (wmax + 3) / 4 * 4 : (wmax + D.lpr - 1) / D.lpr * D.lpr;
    const size_t ne = (size_t)M.n * D.w;
    D.col = c.take<int>(ne);
    D.val = c.take<double>(ne);
    D.val32 = f32 ? c.take<float>(ne) : nullptr;
    const bool packed = pack && D.w % 4 == 0 && D.w <= 16 && D.lpr == 1 && M.m < 65536;
    D.pk = packed ? c.take<uint32_t>((size_t)D.w * M.n) : nullptr;
    D.val16 = half ? c.take<uint16_t>(ne) : nullptr;
    D.pscale = 1.0f;
    return packed;
  };
  for (int l = 0; l < mg.nlev; ++l) {
    const AmgLevel& L = H.lv[l];
    const long n = L.A.n;
    if (l > 0) {
      take_csr(L.A, mg.A[l], 1);
      mg.dinv[l] = c.take<double>(n);
      mg.dinv32[l] = f32 ? c.take<float>(n) : nullptr;
    }
    if (l < mg.nlev - 1) {
      // the restriction from the finest level gathers from the largest vector: a few
      // lanes per row (8 for rows of ~40 entries), each with one batch of entries, keep
      // more of those gathers in flight;
      // the finest-level transfers of an FP32 cycle in FP16 (P packed, R = P^T rounded alike)
      const bool packed = take_csr(L.P, mg.P[l], 1, l == 0 && f16);
      take_csr(L.R, mg.R[l], l == 0 ? 4 : 1, false, packed);
      if (l > 0) {
        take_csr(L.AP, mg.AP[l], 1);
        take_csr(L.RA, mg.RA[l], 1);
      }
    }
    MgVec<double>& v = mg.v64[l];
    v.b = (l > 0) ? c.take<double>(n) : nullptr;
    v.z = (l > 0) ? c.take<double>(n) : nullptr;
    // work vectors of the two-step smoothing (finest level only; the coarser levels keep
    // only their right-hand side b and result z)
    const bool fine = (l == 0 && mg.nlev > 1);
    v.x = fine ? c.take<double>(n) : nullptr;
    v.y = fine ? c.take<double>(n) : nullptr;
    v.d = fine ? c.take<double>(n) : nullptr;
    v.r = fine ? c.take<double>(n) : nullptr;
    MgVec<float>& w = mg.v32[l];
    w = MgVec<float>{};
    if (f32) {
      w.b = (l > 0) ? c.take<float>(n) : nullptr;
      w.z = (l > 0) ? c.take<float>(n) : nullptr;
      w.x = fine ? c.take<float>(n) : nullptr;
      w.y = fine ? c.take<float>(n) : nullptr;
      w.d = fine ? c.take<float>(n) : nullptr;
      w.r = fine ? c.take<float>(n) : nullptr;
    }
    // Chebyshev on [lmin, lmax], lmax = 1.05 rho(D^{-1} A): degree 2 on [lmax/15, lmax] on the
    // finest level, degree 1 (damped Jacobi with weight 1/th) on [lmax/30, lmax] on the
    // coarser ones (intervals chosen by the PCG iteration count they give)
    const double lmax = 1.05 * L.lmax, lmin = lmax / (l == 0 ? 15.0 : 30.0);
    const double th = 0.5 * (lmax + lmin), de = 0.5 * (lmax - lmin);
    const double sig = th / de, rho0 = 1.0 / sig, rho1 = 1.0 / (2.0 * sig - rho0);
    mg.cheb[l] = CheB{th, rho1 * rho0, 2.0 * rho1 / de};
  }
  if (mg.nlev > 0) {
    mg.n_coarse = H.n_coarse;
    mg.coarse_inv = c.take<double>(H.coarse_inv.size());
    mg.coarse_inv32 = f32 ? c.take<float>(H.coarse_inv.size()) : nullptr;
  }
  ctx->ws_need = c.off + 256;
}

extern "C" int dfdg_ctx_workspace_bytes(const dfdg_ctx* cctx, size_t* bytes) {
  if (!cctx || !bytes) return DFDG_E_INVALID_ARG;
  auto* ctx = const_cast<dfdg_ctx*>(cctx);
  if (!ctx->bound) carve(ctx, nullptr);
  *bytes = ctx->ws_need;
  return DFDG_OK;
}

template <typename T>
static hipError_t up(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

extern "C" int dfdg_ctx_bind_workspace(dfdg_ctx* ctx, void* dev, size_t bytes) {
  if (!ctx || !dev) return DFDG_E_INVALID_ARG;
  if (((uintptr_t)dev & 255) != 0) return fail(ctx, DFDG_E_WORKSPACE, "workspace must be 256-byte aligned");
  carve(ctx, nullptr);
  const size_t need = ctx->ws_need;
  if (bytes < need)
    return fail(ctx, DFDG_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  ctx->ws = (char*)dev;
  carve(ctx, ctx->ws);
  if (ctx->ws_need != need) {  // both passes must lay out the same arrays
    ctx->ws = nullptr;
    return fail(ctx, DFDG_E_WORKSPACE, "internal error: workspace layout differs between passes");
  }
  const HostSetup& h = ctx->hs;
  hipStream_t s = ctx->stream;
  HIPC(hipMemsetAsync(ctx->ws, 0, ctx->ws_need - 256, s));
  HIPC(up(const_cast<double*>(ctx->g.Jinv), h.Jinv, s));
  HIPC(up(const_cast<double*>(ctx->g.detJ), h.detJ, s));
  HIPC(up(const_cast<double*>(ctx->g.isq), h.isq, s));
  HIPC(up(const_cast<int*>(ctx->g.nbr), h.nbr, s));
  HIPC(up(const_cast<int*>(ctx->g.code), h.code, s));
  HIPC(up(const_cast<int*>(ctx->g.efacet), h.efacet, s));
  HIPC(up(const_cast<double*>(ctx->g.nx), h.nx, s));
  HIPC(up(const_cast<double*>(ctx->g.ny), h.ny, s));
  if (ctx->g.nz) HIPC(up(const_cast<double*>(ctx->g.nz), h.nz, s));
  HIPC(up(const_cast<double*>(ctx->g.flen), h.flen, s));
  HIPC(up(const_cast<double*>(ctx->g.sig), h.sig, s));
  HIPC(up(const_cast<double*>(ctx->g.sF), h.sF, s));
  HIPC(up(const_cast<double*>(ctx->g.G), h.G, s));
  if (ctx->g.G4) HIPC(up(const_cast<double*>(ctx->g.G4), h.G4, s));
  HIPC(up(const_cast<int*>(ctx->g.qL), h.qL, s));
  HIPC(up(const_cast<int*>(ctx->g.qR), h.qR, s));
  HIPC(up(const_cast<double*>(ctx->g.zdef), h.zdef, s));
  const RefTables& tb = h.tabs;
  HIPC(up(const_cast<double*>(ctx->tb.Vv), tb.Vv, s));
  HIPC(up(const_cast<double*>(ctx->tb.Gv), tb.Gv, s));
  HIPC(up(const_cast<double*>(ctx->tb.Wv), tb.vw, s));
  HIPC(up(const_cast<double*>(ctx->tb.Vf), tb.Vf, s));
  HIPC(up(const_cast<double*>(ctx->tb.Gf), tb.Gf, s));
  HIPC(up(const_cast<double*>(ctx->tb.Wf), tb.fw, s));
  HIPC(up(const_cast<double*>(ctx->tb.Vp), tb.Vp, s));
  HIPC(up(const_cast<double*>(ctx->tb.Wp), tb.pw, s));
  HIPC(up(const_cast<double*>(ctx->tb.Dh), tb.Dh, s));
  HIPC(up(const_cast<double*>(ctx->tb.Ch), tb.Ch, s));
  if (ctx->tb.Zh) HIPC(up(const_cast<double*>(ctx->tb.Zh), tb.Zh, s));
  if (ctx->tb.fpidx) HIPC(up(const_cast<int*>(ctx->tb.fpidx), tb.fpidx, s));
  if (ctx->tb.Qf) HIPC(up(const_cast<double*>(ctx->tb.Qf), tb.Qf, s));
  HIPC(up(const_cast<int*>(ctx->A.cols), h.cols, s));
  HIPC(up(const_cast<double*>(ctx->A.vals), h.vals, s));
  HIPC(up(const_cast<double*>(ctx->A.dinv), h.dinv, s));
  HIPC(up(const_cast<double*>(ctx->A.binv), h.binv, s));
  if (ctx->A.tdef) {  // S D^{-1} z, z = zdef on mode 0 (FP64 on the host)
    const int NS = ctx->A.ns;
    const long E = ctx->E, NF = ctx->NF;
    std::vector<double> t((size_t)E * NF, 0.0);
    for (long F = 0; F < E; ++F)
      for (int sl = 0; sl < NS; ++sl) {
        const long cc = h.cols[(size_t)sl * E + F];
        const double w = h.dinv[(size_t)cc * NF] * h.zdef[cc];
        for (long a = 0; a < NF; ++a) t[(size_t)F * NF + a] += h.vals[(((size_t)sl * NF + a) * NF + 0) * E + F] * w;
      }
    std::vector<float> t32(t.begin(), t.end());
    HIPC(up(const_cast<double*>(ctx->A.tdef), t, s));
    if (ctx->A.tdef32) HIPC(up(const_cast<float*>(ctx->A.tdef32), t32, s));
    HIPC(hipStreamSynchronize(s));  // the host copies end with this block
  }
  if (ctx->A.vals32) {
    std::vector<float> v(h.vals.begin(), h.vals.end()), d(h.dinv.begin(), h.dinv.end()),
        b(h.binv.begin(), h.binv.end());
    HIPC(up(const_cast<float*>(ctx->A.vals32), v, s));
    HIPC(up(const_cast<float*>(ctx->A.dinv32), d, s));
    HIPC(up(const_cast<float*>(ctx->A.binv32), b, s));
    HIPC(hipStreamSynchronize(s));
  }
  if (ctx->A.vals16) {
    double smax = 0;
    for (double v : h.vals) smax = std::max(smax, std::fabs(v));
    if (!(smax > 0)) smax = 1;
    ctx->A.scale16 = (float)smax;
    HIPC(launch_pack_half_pairs(ctx->NF, ctx->A.ns, ctx->E, ctx->A.vals, 1.0 / smax, const_cast<uint32_t*>(ctx->A.vals16),
                                s));
  }
  {
    const bool mixed = ctx->A.vals32 != nullptr;  // FP32 copies were carved
    const AmgHierarchy& H = ctx->H;
    MgDev& mg = ctx->mg;
    std::vector<std::vector<float>> keep;  // float staging buffers stay alive until the sync below
    std::deque<std::vector<double>> keep_d;  // padded copies, likewise
    std::deque<std::vector<int>> keep_i;
    auto f32 = [&](const std::vector<double>& v) -> const std::vector<float>& {
      keep.emplace_back(v.begin(), v.end());
      return keep.back();
    };
    auto up_csr = [&](const Csr& M, DevCsr& D) -> int {
      // padded row-major copy (see DevCsr)
      std::vector<int> ce((size_t)M.n * D.w);
      keep_d.emplace_back((size_t)M.n * D.w, 0.0);
      std::vector<double>& ve = keep_d.back();
      for (int i = 0; i < M.n; ++i) {
        const int b = M.ptr[i], len = M.ptr[i + 1] - b;
        for (int k = 0; k < D.w; ++k) {
          ce[(size_t)i * D.w + k] = len ? M.col[b + std::min(k, len - 1)] : 0;
          if (k < len) ve[(size_t)i * D.w + k] = M.val[b + k];
        }
      }
      keep_i.push_back(std::move(ce));
      HIPC(up(const_cast<int*>(D.col), keep_i.back(), s));
      HIPC(up(const_cast<double*>(D.val), ve, s));
      if (mixed) HIPC(up(const_cast<float*>(D.val32), f32(ve), s));
      if (D.pk || D.val16) {  // the same values in P and R: the same scale and rounding
        double vmax = 0;
        for (double x : ve) vmax = std::max(vmax, std::fabs(x));
        if (!(vmax > 0)) vmax = 1;
        D.pscale = (float)vmax;
        if (D.pk) HIPC(launch_pack_rows(M.n, D.w, D.col, D.val, 1.0 / vmax, const_cast<uint32_t*>(D.pk), s));
        if (D.val16)
          HIPC(launch_to_half((long)ve.size(), D.val, 1.0 / vmax, const_cast<uint16_t*>(D.val16), s));
      }
      return DFDG_OK;
    };
    keep.reserve(8 * kMaxLev + 2);
    for (int l = 0; l < mg.nlev; ++l) {
      const AmgLevel& L = H.lv[l];
      if (l > 0) {
        if (int rc = up_csr(L.A, mg.A[l])) return rc;
        HIPC(up(const_cast<double*>(mg.dinv[l]), L.dinv, s));
        if (mixed) HIPC(up(const_cast<float*>(mg.dinv32[l]), f32(L.dinv), s));
      }
      if (l < mg.nlev - 1) {
        if (int rc = up_csr(L.P, mg.P[l])) return rc;
        if (int rc = up_csr(L.R, mg.R[l])) return rc;
        if (l > 0) {
          if (int rc = up_csr(L.AP, mg.AP[l])) return rc;
          if (int rc = up_csr(L.RA, mg.RA[l])) return rc;
        }
      }
    }
    if (mg.nlev > 0) {
      HIPC(up(const_cast<double*>(mg.coarse_inv), H.coarse_inv, s));
      if (mixed) HIPC(up(const_cast<float*>(mg.coarse_inv32), f32(H.coarse_inv), s));
    }
    HIPC(hipStreamSynchronize(s));
  }
  HIPC(hipStreamSynchronize(s));
  if (!ctx->pinned) HIPC(hipHostMalloc((void**)&ctx->pinned, 4 * sizeof(PcgScalars), hipHostMallocDefault));
  // the device address of the allocation-free diagnostics' scratch on this (current) device
  HIPC(noalloc_scratch(&ctx->noalloc));
  ctx->bound = true;
  for (int i = 0; i < 3; ++i) ctx->hist_count[i] = 0;
  invalidate_guesses(ctx);
  return DFDG_OK;
}

extern "C" const char* dfdg_last_error(const dfdg_ctx* ctx) {
  if (!ctx) return g_mesh_err.c_str();
  return ctx->err.c_str();
}

extern "C" void dfdg_ctx_destroy(dfdg_ctx* ctx) {
  if (!ctx) return;
  for (int j = 0; j < 6; ++j) {
    if (ctx->graph64[j]) (void)hipGraphExecDestroy(ctx->graph64[j]);
    if (ctx->graph32[j]) (void)hipGraphExecDestroy(ctx->graph32[j]);
  }
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->sc_event) (void)hipEventDestroy(ctx->sc_event);
  if (ctx->pinned) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipHostFree(ctx->pinned);
  }
  delete ctx;
}

// ---------------------------------------------------------------------------------------
// facet solve
// ---------------------------------------------------------------------------------------
static int status_of(int done) {
  switch (done) {
    case PCG_CONVERGED: return DFDG_OK;
    case PCG_MAXIT: return DFDG_E_NOT_CONVERGED;
    case PCG_BREAKDOWN: return DFDG_E_BREAKDOWN;
    case PCG_NONFINITE: return DFDG_E_NONFINITE;
    default: return DFDG_E_NOT_CONVERGED;
  }
}

static int extrapolate_into(dfdg_ctx* ctx, int s, double* out);

// Copies the scalars to the host and waits for them.  When a forward stage's start value
// is due (defer_slot), its kernels are enqueued behind the copy, so that the GPU forms it
// while the host reads the scalars and enqueues the next work.
static int read_scalars(dfdg_ctx* ctx, PcgScalars* dev, PcgScalars& out) {
  HIPC(hipMemcpyAsync(ctx->pinned, dev, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
  const int d = ctx->defer_slot;
  if (d >= 0) {
    ctx->defer_slot = -1;
    if (!ctx->sc_event) HIPC(hipEventCreateWithFlags(&ctx->sc_event, hipEventDisableTiming));
    HIPC(hipEventRecord(ctx->sc_event, ctx->stream));
    const int rc = extrapolate_into(ctx, d, ctx->gbuf[d]);
    if (rc) return rc;
    ctx->gready[d] = true;
    HIPC(hipEventSynchronize(ctx->sc_event));
  } else {
    HIPC(hipStreamSynchronize(ctx->stream));
  }
  out = *ctx->pinned;
  return DFDG_OK;
}

// Capture one PCG iteration of the given parity (the buffer and partial-slot choice
// alternates between odd and even iterations and is part of the launch arguments; the
// iteration index itself is read by the kernels from the device scalars).
template <typename Step>
static int capture_iteration(dfdg_ctx* ctx, int parity, int count, Step step, hipGraphExec_t* out) {
  if (!ctx->cap_stream) HIPC(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  HIPC(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
  hipError_t e = hipSuccess;
  for (int i = 0; i < count && e == hipSuccess; ++i) e = step(((parity + i) & 1) ? 1 : 2, ctx->cap_stream);
  if (e != hipSuccess) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(ctx->cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    return fail(ctx, DFDG_E_HIP, std::string("PCG capture: ") + hipGetErrorString(e));
  }
  hipGraph_t g = nullptr;
  HIPC(hipStreamEndCapture(ctx->cap_stream, &g));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(ctx, DFDG_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  return DFDG_OK;
}

// Run PCG iterations (already initialised on the device) until the device flags an end.
// The host enqueues chunks of iterations (graph replays or eager launches) and reads the
// scalars after each chunk.  The first chunk is the length of the previous run (*hint);
// later chunks follow the mean contraction of (r, r) observed so far, so that few
// iterations run past the end (those exit at their first instruction).
template <typename Step>
static int pcg_loop(dfdg_ctx* ctx, PcgScalars* sc, int maxit, Step step, hipGraphExec_t (&graph)[6], int* hint,
                    PcgScalars& fin) {
  // the first chunk is enqueued right after the initialisation, without reading the
  // scalars first (a run that is already over, e.g. for a zero right-hand side, makes those
  // launches return at once), so the GPU does not wait for a host round trip
  int rc = DFDG_OK;
  const bool use_graph = ctx->prm.graphs != 0;
  if (use_graph)
    for (int j = 0; j < 6; ++j)
      if (!graph[j]) {
        rc = capture_iteration(ctx, j & 1, 1 << (j >> 1), step, &graph[j]);
        if (rc) return rc;
      }
  const bool amg = ctx->prm.precond == DFDG_AMG;
  // With the multigrid cycle (two levels or more) the last kernel of an iteration applies
  // the stopping test, so a run of n iterations takes n launches; otherwise the next
  // iteration's first kernel applies it and a run takes n + 1
  const int extra = (amg && ctx->mg.nlev >= 2) ? 0 : 1;
  // the first chunk: the fewest iterations among the last kHintRuns runs.  With start
  // values that vary in quality the count varies from solve to solve; a chunk that falls
  // short costs one host round trip, while each iteration enqueued past the end still runs
  // the multigrid cycle's loads (its kernels test the stop flag only before their stores)
  int h = hint[0];
  for (int j = 1; j < kHintRuns; ++j)
    if (hint[j] > 0) h = std::min(h, hint[j]);
  int chunk = h > 0 ? h + extra : (amg ? 16 : 64);
  fin.done = PCG_RUNNING;
  int launched = 0;
  while (fin.done == PCG_RUNNING) {
    for (int c = 0; c < chunk;) {
      const int it = launched + 1 + c;
      if (use_graph) {  // groups of 4 or 2 iterations where the chunk allows (fewer graph launches)
        const int j = chunk - c >= 4 ? 2 : (chunk - c >= 2 ? 1 : 0);
        HIPC(hipGraphLaunch(graph[2 * j + (it & 1)], ctx->stream));
        c += 1 << j;
      } else {
        hipError_t e = step(it, ctx->stream);
        if (e != hipSuccess) return fail(ctx, DFDG_E_HIP, std::string("PCG launch: ") + hipGetErrorString(e));
        ++c;
      }
    }
    launched += chunk;
    rc = read_scalars(ctx, sc, fin);
    if (rc) return rc;
    if (fin.done != PCG_RUNNING) break;
    if (launched > maxit + 2) return fail(ctx, DFDG_E_NOT_CONVERGED, "PCG did not stop at its iteration limit");
    // fin.rr is (r, r) after launched - 1 iterations; one more iteration has run and one
    // further launch applies the test, so the estimate from fin.rr counts both
    int next = std::max(chunk / 2, 2);
    if (fin.iters > 0 && fin.rr > 0 && fin.rr0 > fin.rr && fin.tol2 > 0) {
      const double rate = std::log(fin.rr / fin.rr0) / fin.iters;  // < 0
      next = (int)std::ceil(std::log(fin.tol2 / fin.rr) / rate);
    }
    chunk = std::min(std::max(next, 1), 1024);
  }
  for (int j = kHintRuns - 1; j > 0; --j) hint[j] = hint[j - 1];
  hint[0] = fin.iters;
  return DFDG_OK;
}

// ---- start values projected onto earlier forward stage solutions ----------------------
static PjVecs pj_vecs(double* const* v, int n) {
  PjVecs p{};
  for (int i = 0; i < n; ++i) p.p[i] = v[i];
  return p;
}

// x = the element of span X closest in the S-norm to the solution of S x = g (g in ctx->gv);
// also kept in pjx0, with its coefficients on the stored vectors in pjcA, for proj_push.
static int proj_start(dfdg_ctx* ctx, double* x) {
  hipStream_t s = ctx->stream;
  const long n = ctx->nL;
  const int nb = ctx->proj_nb;
  if (nb == 0) {
    HIPC(launch_fill(n, 0.0, x, s));
    return DFDG_OK;
  }
  const PjVecs B = pj_vecs(ctx->pjX, nb);
  HIPC(launch_pj_dots(n, nb, B, ctx->gv, ctx->pjpart, s));
  HIPC(launch_pj_small(n, nb, 0, ctx->pjpart, ctx->pjT, ctx->pjnrm, ctx->pjcA, s));
  HIPC(launch_pj_combine(n, nb, B, ctx->pjcA, x, ctx->pjx0, s));
  return DFDG_OK;
}

// Basis vector `slot` from the solution a of S a = Sa (Sa its right-hand side): the part of
// a S-orthogonal to X_0..X_{slot-1}.  First Gram-Schmidt pass on the vectors (with the
// start value's coefficients when a0 = the start value is given: a - a0 is then that part
// up to rounding), second pass as a column of T.  ca, cSa (optional) receive copies of a, Sa.
static int proj_add(dfdg_ctx* ctx, int slot, const double* a, const double* a0, const double* Sa, double* ca,
                    double* cSa) {
  hipStream_t s = ctx->stream;
  const long n = ctx->nL;
  const PjVecs B = pj_vecs(ctx->pjX, slot), SB = pj_vecs(ctx->pjSX, slot);
  const double* w = ctx->pjcA;
  if (slot > 0 && !a0) {
    HIPC(launch_pj_dots(n, slot, B, Sa, ctx->pjpart, s));
    HIPC(launch_pj_small(n, slot, 0, ctx->pjpart, ctx->pjT, ctx->pjnrm, ctx->pjcB, s));
    w = ctx->pjcB;
  }
  HIPC(launch_pj_update(n, slot, B, SB, w, a, a0, Sa, ctx->pjX[slot], ctx->pjSX[slot], ca, cSa, ctx->pjpart, s));
  HIPC(launch_pj_small(n, slot, 1, ctx->pjpart, ctx->pjT, ctx->pjnrm, nullptr, s));
  return DFDG_OK;
}

// After a converged forward stage solve with solution x (start value from proj_start, the
// right-hand side in ctx->gv): keep (x, g) in the ring, and extend the basis, or rebuild it
// from the ring (oldest first) when it is full.
static int proj_push(dfdg_ctx* ctx, const double* x) {
  hipStream_t s = ctx->stream;
  const int h = ctx->proj_head;
  ctx->proj_head = (h + 1) % kProjKeep;
  ctx->proj_raw = std::min(ctx->proj_raw + 1, kProjKeep);
  if (ctx->proj_nb < kProjMax) {
    const int slot = ctx->proj_nb;
    const int rc = proj_add(ctx, slot, x, slot > 0 ? ctx->pjx0 : nullptr, ctx->gv, ctx->pjRawL[h], ctx->pjRawG[h]);
    if (!rc) ctx->proj_nb = slot + 1;
    return rc;
  }
  const size_t bytes = (size_t)ctx->nL * sizeof(double);
  HIPC(hipMemcpyAsync(ctx->pjRawL[h], x, bytes, hipMemcpyDeviceToDevice, s));
  HIPC(hipMemcpyAsync(ctx->pjRawG[h], ctx->gv, bytes, hipMemcpyDeviceToDevice, s));
  ctx->proj_nb = 0;
  int rc = DFDG_OK;
  for (int j = 0; j < ctx->proj_raw && !rc; ++j) {
    const int r = (ctx->proj_head - ctx->proj_raw + j + kProjKeep) % kProjKeep;
    rc = proj_add(ctx, j, ctx->pjRawL[r], nullptr, ctx->pjRawG[r], nullptr, nullptr);
    if (!rc) ctx->proj_nb = j + 1;
  }
  return rc;
}

// Solve S lam = g for the q currently in ctx->q; lam holds the start on entry.  The PCG
// runs in the fixed buffer lamx (captured graphs keep their arguments).
static int solve_facets(dfdg_ctx* ctx, double* lam, dfdg_solve_info* info, const double** sol = nullptr) {
  const int NF = ctx->NF;
  const bool bj = ctx->prm.precond == DFDG_BLOCK_JACOBI;
  hipStream_t s = ctx->stream;
  const DevGeo& g = ctx->g;
  const DevBsr& A = ctx->A;
  double* x = ctx->lamx;
  // a forward stage solve with projected start values forms its start once g is known
  const bool proj = ctx->proj_on && ctx->proj_req && ctx->prm.precision == DFDG_FP64;
  if (lam != x && !proj) HIPC(hipMemcpyAsync(x, lam, ctx->nL * sizeof(double), hipMemcpyDeviceToDevice, s));
  PcgScalars fin{};
  dfdg_solve_info inf{};
  const bool amg = ctx->prm.precond == DFDG_AMG;
  const int pc = amg ? 2 : (bj ? 1 : 0);
  // the FP64 PCG: the FP64 path, and the mixed form's Krylov refinement (mixed_solver = 1),
  // whose FP64 outer iterations refine to ir_rtol with the FP32 multigrid cycle as the inner
  // FP32 work
  const bool krylov = ctx->prm.precision == DFDG_FP64 || ctx->prm.mixed_solver == 1;
  if (krylov) {
    const PcgBufs& pb = ctx->pb;
    const bool mixed = ctx->prm.precision == DFDG_MIXED;
    HIPC(launch_gather_g(NF, g, ctx->q, ctx->gv, pb, mixed ? ctx->prm.ir_rtol : ctx->prm.cg_rtol, ctx->prm.cg_maxit, s));
    if (proj) {
      const int rc = proj_start(ctx, x);
      if (rc) return rc;
    }
    HIPC(launch_pcg_init(NF, bj, g, A, ctx->gv, x, ctx->r, ctx->z, ctx->p[0], pb, s, !proj));
    const bool c32 = mixed || ctx->prm.mg_fp32 != 0;
    const bool fused = amg && ctx->mg.nlev >= 2;
    if (amg) {
      if (c32) HIPC((launch_vcycle<float, double>(NF, g, A, ctx->mg, ctx->r, ctx->z, pb.rz[0], pb.sc, s)));
      else HIPC((launch_vcycle<double, double>(NF, g, A, ctx->mg, ctx->r, ctx->z, pb.rz[0], pb.sc, s)));
    }
    auto step = [&](int it, hipStream_t st) -> hipError_t {
      double* pin = ctx->p[(it - 1) & 1];
      double* pout = ctx->p[it & 1];
      if (fused) {  // residual alternates between r (even iterations) and rb (odd)
        double* rin = (it & 1) ? ctx->r : ctx->rb;
        double* rout = (it & 1) ? ctx->rb : ctx->r;
        if (c32)
          return launch_pcg_iteration_mg<float, double>(NF, g, A, ctx->mg, pb, it, ctx->z, pin, pout, ctx->Sp, x,
                                                        rin, rout, ctx->z, st);
        return launch_pcg_iteration_mg<double, double>(NF, g, A, ctx->mg, pb, it, ctx->z, pin, pout, ctx->Sp, x, rin,
                                                       rout, ctx->z, st);
      }
      hipError_t e = launch_pcg_spmv(NF, g, A, ctx->z, pin, pout, ctx->Sp, pb, it, st);
      if (e != hipSuccess) return e;
      e = launch_pcg_update(NF, pc, g, A, pout, ctx->Sp, x, ctx->r, ctx->z, pb, it, st);
      if (e != hipSuccess || !amg) return e;
      if (c32) return launch_vcycle<float, double>(NF, g, A, ctx->mg, ctx->r, ctx->z, pb.rz[it & 1], pb.sc, st);
      return launch_vcycle<double, double>(NF, g, A, ctx->mg, ctx->r, ctx->z, pb.rz[it & 1], pb.sc, st);
    };
    int rc = pcg_loop(ctx, pb.sc, ctx->prm.cg_maxit, step, ctx->graph64, ctx->iters_hint[0], fin);
    if (rc) return rc;
    inf.iterations = fin.iters;
    inf.refinements = mixed ? fin.iters : 0;  // each outer FP64 iteration refines once
    inf.rel_residual = fin.gg > 0 ? std::sqrt(std::max(fin.rr, 0.0) / fin.gg) : 0.0;
    inf.initial_rel_residual = (fin.gg > 0 && !fin.zero_rhs) ? std::sqrt(std::max(fin.rr0, 0.0) / fin.gg) : 0.0;
    inf.status = status_of(fin.done);
  } else {
    // mixed: FP64 refinement around FP32 inner PCG (S in FP32), FP64 residuals
    const PcgBufs& pb = ctx->pb;
    const PcgBufs& pi = ctx->pb32;
    const double inner = ctx->prm.inner_rtol;
    HIPC(launch_gather_g(NF, g, ctx->q, ctx->gv, pb, ctx->prm.ir_rtol, ctx->prm.cg_maxit, s));
    HIPC(launch_ir_residual(NF, g, A, ctx->gv, x, nullptr, 0, ctx->r64, pb, pi.sc, inner, ctx->prm.cg_maxit, s));
    PcgScalars o{};
    int rc = read_scalars(ctx, pb.sc, o);
    if (rc) return rc;
    if (o.zero_rhs) HIPC(launch_fill(ctx->nL, 0.0, x, s));  // right-hand side at rounding level
    inf.initial_rel_residual = (o.gg > 0 && !o.zero_rhs) ? std::sqrt(std::max(o.rr, 0.0) / o.gg) : 0.0;
    int total = 0, nref = 0, st = DFDG_OK;
    const bool fused = amg && ctx->mg.nlev >= 2;
    auto step = [&](int it, hipStream_t sm) -> hipError_t {
      float* pin = ctx->p32[(it - 1) & 1];
      float* pout = ctx->p32[it & 1];
      if (fused) {
        float* rin = (it & 1) ? ctx->r32 : ctx->r32b;
        float* rout = (it & 1) ? ctx->r32b : ctx->r32;
        return launch_pcg_iteration_mg<float, float>(NF, g, A, ctx->mg, pi, it, ctx->z32, pin, pout, ctx->Sp32,
                                                     ctx->x32, rin, rout, ctx->z32, sm);
      }
      hipError_t e = launch_pcg32_spmv(NF, g, A, ctx->z32, pin, pout, ctx->Sp32, pi, it, sm);
      if (e != hipSuccess) return e;
      e = launch_pcg32_update(NF, pc, g, A, pout, ctx->Sp32, ctx->x32, ctx->r32, ctx->z32, pi, it, sm);
      if (e != hipSuccess || !amg) return e;
      return launch_vcycle<float, float>(NF, g, A, ctx->mg, ctx->r32, ctx->z32, pi.rz[it & 1], pi.sc, sm);
    };
    while (!o.zero_rhs && o.rr > o.tol2) {
      if (nref >= 30 || total >= ctx->prm.cg_maxit) { st = DFDG_E_NOT_CONVERGED; break; }
      HIPC(launch_pcg32_init(NF, bj, g, A, ctx->r64, ctx->x32, ctx->r32, ctx->z32, ctx->p32[0], pi, s));
      if (amg) HIPC((launch_vcycle<float, float>(NF, g, A, ctx->mg, ctx->r32, ctx->z32, pi.rz[0], pi.sc, s)));
      rc = pcg_loop(ctx, pi.sc, ctx->prm.cg_maxit - total, step, ctx->graph32, ctx->iters_hint[1], fin);
      if (rc) return rc;
      total += fin.iters;
      ++nref;
      // an inner run that meets (p, S p) <= 0 in FP32 (rounding near the null space of S)
      // after some progress ends with its last iterate; the FP64 refinement residual
      // decides whether more is needed
      if (fin.done == PCG_NONFINITE || (fin.done == PCG_BREAKDOWN && fin.iters < 1)) st = status_of(fin.done);
      // the next inner run may take what is left of the iteration limit, so that the device
      // stops it before the host guard of pcg_loop would
      HIPC(launch_ir_residual(NF, g, A, ctx->gv, x, ctx->x32, 1, ctx->r64, pb, pi.sc, inner,
                              std::max(1, ctx->prm.cg_maxit - total), s));
      rc = read_scalars(ctx, pb.sc, o);
      if (rc) return rc;
      if (st != DFDG_OK) break;
      if (!std::isfinite(o.rr)) { st = DFDG_E_NONFINITE; break; }
    }
    inf.iterations = total;
    inf.refinements = nref;
    inf.rel_residual = o.gg > 0 ? std::sqrt(std::max(o.rr, 0.0) / o.gg) : 0.0;
    inf.status = st;
  }
  // the multiplier is fixed up to the kernel of S: keep the representative orthogonal to
  // it, so that warm starts built from earlier solutions cannot let it drift
  HIPC(launch_deflate(NF, g, x, ctx->pb.gg, s));
  // a projected solve leaves its multiplier in lamx (*sol), which nothing overwrites before
  // the recovery reads it
  if (lam != x && !proj) HIPC(hipMemcpyAsync(lam, x, ctx->nL * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (sol) *sol = proj ? x : lam;
  if (proj && inf.status == DFDG_OK && !fin.zero_rhs) {
    const int rc = proj_push(ctx, x);
    if (rc) return rc;
  }
  if (info) *info = inf;
  return DFDG_OK;
}

static int mass_solve_impl(dfdg_ctx* ctx, const void* F, bool f32, double* U, double* lam, bool cold,
                           dfdg_solve_info* info, int mode, double ca, const double* Un, double cb,
                           const double* Us, double dt) {
  hipStream_t s = ctx->stream;
  HIPC(el_cond_rhs(ctx, f32, F, s));
  if (cold) HIPC(launch_fill(ctx->nL, 0.0, lam, s));
  dfdg_solve_info inf{};
  const double* sol = lam;
  int rc = solve_facets(ctx, lam, &inf, &sol);
  if (rc) return rc;
  HIPC(el_recover(ctx, f32, F, sol, U, mode, ca, Un, cb, Us, dt, s));
  if (info) *info = inf;
  return DFDG_OK;
}

// ---------------------------------------------------------------------------------------
// public hot-path entry points
// ---------------------------------------------------------------------------------------
extern "C" int dfdg_proj_rule(const dfdg_ctx* ctx, double* pts, double* w) {
  if (!ctx || !pts || !w) return DFDG_E_INVALID_ARG;
  std::memcpy(pts, ctx->hs.tabs.pq.data(), ctx->hs.tabs.pq.size() * sizeof(double));
  std::memcpy(w, ctx->hs.tabs.pw.data(), ctx->hs.tabs.pw.size() * sizeof(double));
  return DFDG_OK;
}

extern "C" int dfdg_load_vector(dfdg_ctx* ctx, const double* fq, double* F) {
  NEED_BOUND(ctx);
  if (!fq || !F) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  HIPC(el_load_vector(ctx, fq, F, ctx->stream));
  return DFDG_OK;
}

extern "C" int dfdg_hdiv_mass_solve(dfdg_ctx* ctx, const double* F, double* U, double* lam_io,
                                    dfdg_solve_info* info) {
  NEED_BOUND(ctx);
  if (!F || !U) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  double* lam = lam_io ? lam_io : ctx->lamw;
  dfdg_solve_info inf{};
  int rc = mass_solve_impl(ctx, F, false, U, lam, lam_io == nullptr, &inf, 0, 0, nullptr, 0, nullptr, 0);
  if (rc) return rc;
  if (info) *info = inf;
  if (inf.status != DFDG_OK) return fail(ctx, inf.status, "facet PCG did not converge");
  return DFDG_OK;
}

extern "C" int dfdg_project(dfdg_ctx* ctx, const double* fq, double* U, dfdg_solve_info* info) {
  NEED_BOUND(ctx);
  if (!fq || !U) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  HIPC(el_load_vector(ctx, fq, ctx->Lbuf, ctx->stream));
  dfdg_solve_info inf{};
  int rc = mass_solve_impl(ctx, ctx->Lbuf, false, U, ctx->lamw, true, &inf, 0, 0, nullptr, 0, nullptr, 0);
  if (rc) return rc;
  if (info) *info = inf;
  if (inf.status != DFDG_OK) return fail(ctx, inf.status, "facet PCG did not converge");
  return DFDG_OK;
}

extern "C" int dfdg_dg_residual(dfdg_ctx* ctx, const double* U, double* L) {
  NEED_BOUND(ctx);
  if (!U || !L) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  HIPC(el_residual(ctx, false, U, L, ctx->stream));
  return DFDG_OK;
}

extern "C" int dfdg_reset_history(dfdg_ctx* ctx) {
  if (!ctx) return DFDG_E_INVALID_ARG;
  for (int i = 0; i < 3; ++i) ctx->hist_count[i] = 0;
  ctx->hist_count[6] = 0;
  invalidate_guesses(ctx);
  return DFDG_OK;
}

// The forward history belongs to one integrator; switching starts from an empty one.
static void use_integrator(dfdg_ctx* ctx, int id) {
  if (ctx->integrator != id) {
    for (int i = 0; i < 3; ++i) ctx->hist_count[i] = 0;
    ctx->hist_count[6] = 0;
    invalidate_guesses(ctx);
    ctx->integrator = id;
  }
}

extern "C" int dfdg_reset_adjoint_history(dfdg_ctx* ctx) {
  if (!ctx) return DFDG_E_INVALID_ARG;
  for (int i = 3; i < 6; ++i) ctx->hist_count[i] = 0;
  return DFDG_OK;
}

extern "C" int dfdg_history_bytes(const dfdg_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return DFDG_E_INVALID_ARG;
  *bytes = (size_t)3 * kHistDepth * ctx->nL * sizeof(double);
  return DFDG_OK;
}

// Blob layout: [3 stages][kHistDepth][nL], newest first.
extern "C" int dfdg_history_save(dfdg_ctx* ctx, double* hist, int* counts) {
  NEED_BOUND(ctx);
  if (!hist || !counts) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  const size_t nL = ctx->nL, nb = nL * sizeof(double);
  for (int st = 0; st < 3; ++st) {
    counts[st] = ctx->hist_count[st];
    for (int j = 0; j < ctx->hist_count[st]; ++j)
      HIPC(hipMemcpyAsync(hist + (size_t)(kHistDepth * st + j) * nL, ctx->hist[st][j], nb, hipMemcpyDeviceToDevice,
                          ctx->stream));
  }
  return DFDG_OK;
}

extern "C" int dfdg_history_restore(dfdg_ctx* ctx, const double* hist, const int* counts) {
  NEED_BOUND(ctx);
  if (!hist || !counts) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  for (int st = 0; st < 3; ++st)
    if (counts[st] < 0 || counts[st] > kHistDepth) return fail(ctx, DFDG_E_INVALID_ARG, "history counts must be in 0..6");
  const size_t nL = ctx->nL, nb = nL * sizeof(double);
  for (int st = 0; st < 3; ++st) {
    for (int j = 0; j < counts[st]; ++j)
      HIPC(hipMemcpyAsync(ctx->hist[st][j], hist + (size_t)(kHistDepth * st + j) * nL, nb, hipMemcpyDeviceToDevice,
                          ctx->stream));
    ctx->hist_count[st] = counts[st];
  }
  invalidate_guesses(ctx);
  ctx->integrator = 1;
  return DFDG_OK;
}

// Start value of the next facet solve of history slot s (which has kept multipliers) into out.
static int extrapolate_into(dfdg_ctx* ctx, int s, double* out) {
  const int n = ctx->hist_count[s];
  HistPtrs h;
  for (int j = 0; j < kHistDepth; ++j) h.p[j] = ctx->hist[s][j];
  if (ctx->prm.extrapolate == kExtrapAdaptive) {
    const int omax = std::min(4, n - 2);  // a backtest of order o needs o + 2 multipliers
    if (omax >= 1) {
      HIPC(launch_extrapolate_adaptive(ctx->nL, omax, h, ctx->xpart, out, ctx->stream));
      return DFDG_OK;
    }
  }
  const int order = std::min(std::min(ctx->prm.extrapolate, 4), n - 1);
  HIPC(launch_extrapolate(ctx->nL, order, h, out, ctx->stream));
  return DFDG_OK;
}

// Start value (in lamw) of the facet solve of history slot s; returns whether it is a cold
// start.  A forward stage's value formed ahead (gbuf) is taken over by exchanging buffers:
// it was formed from the same history, after that slot's last update.
static int stage_guess(dfdg_ctx* ctx, int s, bool* cold) {
  const int n = ctx->hist_count[s];
  *cold = (n == 0);
  if (n == 0) return DFDG_OK;
  if (s < 3 && ctx->gready[s]) {
    std::swap(ctx->lamw, ctx->gbuf[s]);
    ctx->gready[s] = false;
    return DFDG_OK;
  }
  return extrapolate_into(ctx, s, ctx->lamw);
}
static void stage_push(dfdg_ctx* ctx, int s) {
  double* old = ctx->hist[s][kHistDepth - 1];
  for (int j = kHistDepth - 1; j > 0; --j) ctx->hist[s][j] = ctx->hist[s][j - 1];
  ctx->hist[s][0] = ctx->lamw;
  ctx->lamw = old;
  ctx->hist_count[s] = std::min(ctx->hist_count[s] + 1, kHistDepth);
}

// One stage: out = a Un + b (Us + dt M^{-1} L(Us)).
static int rk_stage(dfdg_ctx* ctx, int s, const double* Us, const double* Un, double a, double b, double dt,
                    double* out, dfdg_solve_info* inf) {
  const bool mixed = ctx->prm.precision == DFDG_MIXED;
  void* L = mixed ? (void*)ctx->L32 : (void*)ctx->Lbuf;
  HIPC(el_residual(ctx, mixed, Us, L, ctx->stream));
  if (ctx->proj_on) {  // start value projected inside the solve, once its right-hand side is known
    ctx->proj_req = true;
    const int rc = mass_solve_impl(ctx, L, mixed, out, ctx->lamw, false, inf, 1, a, Un, b, Us, dt);
    ctx->proj_req = false;
    return rc;
  }
  bool cold;
  int rc = stage_guess(ctx, s, &cold);
  if (rc) return rc;
  // the next forward stage's start value, formed while the host waits for this solve
  const int next = (s + 1) % 3;
  if (ctx->hist_count[next] > 0 && !ctx->gready[next]) ctx->defer_slot = next;
  rc = mass_solve_impl(ctx, L, mixed, out, ctx->lamw, cold, inf, 1, a, Un, b, Us, dt);
  ctx->defer_slot = -1;
  if (rc) return rc;
  stage_push(ctx, s);
  return DFDG_OK;
}

// Shu-Osher TVD-RK3 (eq. (rk3)), each bracket u + dt M^{-1} L(u) done by one solve; the
// states entering stages 1 and 2 are left in U1 and U2.
static int rk3_core(dfdg_ctx* ctx, double* U, double dt, double* U1, double* U2, dfdg_step_info* info) {
  dfdg_step_info st{};
  dfdg_solve_info si[3];
  int rc = rk_stage(ctx, 0, U, U, 0.0, 1.0, dt, U1, &si[0]);
  if (!rc) rc = rk_stage(ctx, 1, U1, U, 0.75, 0.25, dt, U2, &si[1]);
  if (!rc) rc = rk_stage(ctx, 2, U2, U, 1.0 / 3.0, 2.0 / 3.0, dt, U, &si[2]);
  if (rc) return rc;
  st.status = DFDG_OK;
  for (int s = 0; s < 3; ++s) {
    st.iterations[s] = si[s].iterations;
    st.initial_rel_residual[s] = si[s].initial_rel_residual;
    st.max_refinements = std::max(st.max_refinements, si[s].refinements);
    st.max_rel_residual = std::max(st.max_rel_residual, si[s].rel_residual);
    if (si[s].status != DFDG_OK) st.status = si[s].status;
  }
  if (info) *info = st;
  if (st.status != DFDG_OK) return fail(ctx, st.status, "a stage's facet solve did not converge");
  return DFDG_OK;
}

extern "C" int dfdg_rk3_step(dfdg_ctx* ctx, double* U, double dt, dfdg_step_info* info) {
  NEED_BOUND(ctx);
  if (!U) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, DFDG_E_INVALID_ARG, "dt must be finite and > 0");
  use_integrator(ctx, 1);
  return rk3_core(ctx, U, dt, ctx->Ustage, ctx->Ustage, info);
}

// out = M^{-1} L(Us), warm-started from history slot s (one stage of RK4).
static int pl_stage(dfdg_ctx* ctx, int s, const double* Us, double* out, dfdg_solve_info* inf) {
  const bool mixed = ctx->prm.precision == DFDG_MIXED;
  void* L = mixed ? (void*)ctx->L32 : (void*)ctx->Lbuf;
  HIPC(el_residual(ctx, mixed, Us, L, ctx->stream));
  if (ctx->proj_on) {
    ctx->proj_req = true;
    const int rc = mass_solve_impl(ctx, L, mixed, out, ctx->lamw, false, inf, 0, 0, nullptr, 0, nullptr, 0);
    ctx->proj_req = false;
    return rc;
  }
  bool cold;
  int rc = stage_guess(ctx, s, &cold);
  if (rc) return rc;
  rc = mass_solve_impl(ctx, L, mixed, out, ctx->lamw, cold, inf, 0, 0, nullptr, 0, nullptr, 0);
  if (rc) return rc;
  stage_push(ctx, s);
  return DFDG_OK;
}

extern "C" int dfdg_rk4_step(dfdg_ctx* ctx, double* U, double dt, dfdg_rk4_info* info) {
  NEED_BOUND(ctx);
  if (!U) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, DFDG_E_INVALID_ARG, "dt must be finite and > 0");
  use_integrator(ctx, 2);
  hipStream_t s = ctx->stream;
  const long n = ctx->nU;
  const size_t nb = n * sizeof(double);
  double* K[4] = {ctx->Ustages[0], ctx->Ustages[1], ctx->Ustages[2], ctx->Ybar};
  double* Ui = ctx->Wbuf;
  const int slot[4] = {0, 1, 2, 6};
  const double c[4] = {0.5, 0.5, 1.0, 0.0};  // u_{i+1} = u^n + c_i dt k_i
  dfdg_solve_info si[4]{};
  const double* Us = U;
  for (int i = 0; i < 4; ++i) {
    int rc = pl_stage(ctx, slot[i], Us, K[i], &si[i]);
    if (rc) return rc;
    if (i < 3) {
      HIPC(hipMemcpyAsync(Ui, U, nb, hipMemcpyDeviceToDevice, s));
      HIPC(launch_axpby(n, c[i] * dt, K[i], 1.0, Ui, s));
      Us = Ui;
    }
  }
  // u^{n+1} = u^n + dt/6 (k1 + 2 k2 + 2 k3 + k4)
  const double w[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
  for (int i = 0; i < 4; ++i) HIPC(launch_axpby(n, w[i], K[i], 1.0, U, s));
  dfdg_rk4_info st{};
  st.status = DFDG_OK;
  for (int i = 0; i < 4; ++i) {
    st.iterations[i] = si[i].iterations;
    st.max_rel_residual = std::max(st.max_rel_residual, si[i].rel_residual);
    if (si[i].status != DFDG_OK) st.status = si[i].status;
  }
  if (info) *info = st;
  if (st.status != DFDG_OK) return fail(ctx, st.status, "a stage's facet solve did not converge");
  return DFDG_OK;
}

extern "C" int dfdg_fe_step(dfdg_ctx* ctx, double* U, double dt, dfdg_solve_info* info) {
  NEED_BOUND(ctx);
  if (!U) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, DFDG_E_INVALID_ARG, "dt must be finite and > 0");
  use_integrator(ctx, 3);
  dfdg_solve_info inf{};
  int rc = rk_stage(ctx, 0, U, U, 0.0, 1.0, dt, U, &inf);  // U <- U + dt M^{-1} L(U)
  if (rc) return rc;
  if (info) *info = inf;
  if (inf.status != DFDG_OK) return fail(ctx, inf.status, "the facet solve did not converge");
  return DFDG_OK;
}

extern "C" int dfdg_rk3_step_stages(dfdg_ctx* ctx, double* U, double dt, double* U1, double* U2,
                                    dfdg_step_info* info) {
  NEED_BOUND(ctx);
  if (!U || !U1 || !U2) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (U1 == U || U2 == U || U1 == U2) return fail(ctx, DFDG_E_INVALID_ARG, "U, U1 and U2 must be distinct buffers");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, DFDG_E_INVALID_ARG, "dt must be finite and > 0");
  use_integrator(ctx, 1);
  return rk3_core(ctx, U, dt, U1, U2, info);
}

// ---------------------------------------------------------------------------------------
// adjoint form
// ---------------------------------------------------------------------------------------
static hipError_t residual_vjp(dfdg_ctx* ctx, const double* U, const double* Lbar, double* Ubar, hipStream_t s) {
  if (ctx->dim == 3) return launch_residual_vjp3(ctx->K, ctx->g, ctx->tb, U, Lbar, Ubar, ctx->prm.nu, s);
  return launch_residual_vjp(ctx->K, ctx->g, ctx->tb, U, Lbar, Ubar, ctx->prm.nu, s);
}

extern "C" int dfdg_dg_residual_vjp(dfdg_ctx* ctx, const double* U, const double* Lbar, double* Ubar) {
  NEED_BOUND(ctx);
  if (!U || !Lbar || !Ubar) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  HIPC(residual_vjp(ctx, U, Lbar, Ubar, ctx->stream));
  return DFDG_OK;
}

// Reverse of dfdg_rk3_step.  With FE(u) = u + dt P L(u), P the mass solve (symmetric):
//   U1 = FE(Un),  U2 = 3/4 Un + 1/4 FE(U1),  U3 = 1/3 Un + 2/3 FE(U2),
// and J_FE(u)^T y = y + dt J_L(u)^T P y.  Given Y3 = Ubar_{n+1}:
//   Y2 = 2/3 J_FE(U2)^T Y3,  Y1 = 1/4 J_FE(U1)^T Y2,
//   Ubar_n = 1/3 Y3 + 3/4 Y2 + J_FE(Un)^T Y1.
static int fe_transpose(dfdg_ctx* ctx, int stage, const double* u, const double* y, double* out, double dt,
                        dfdg_solve_info* si) {
  hipStream_t s = ctx->stream;
  // P y, warm-started from the same stage's adjoint solves of the steps processed before
  bool cold;
  int rc = stage_guess(ctx, 3 + stage, &cold);
  if (rc) return rc;
  rc = mass_solve_impl(ctx, y, false, ctx->Wbuf, ctx->lamw, cold, si, 0, 0, nullptr, 0, nullptr, 0);
  if (rc) return rc;
  stage_push(ctx, 3 + stage);
  HIPC(residual_vjp(ctx, u, ctx->Wbuf, out, s));
  HIPC(launch_axpby(ctx->nU, 1.0, y, dt, out, s));  // out = y + dt J^T P y
  return DFDG_OK;
}

// Reverse sweep of one TVD-RK3 step given its stage states U^n, U1, U2; Ybar in place.
static int rk3_vjp_core(dfdg_ctx* ctx, const double* Un, const double* U1, const double* U2, double* Ybar,
                        double dt, dfdg_solve_info (&si)[3]) {
  hipStream_t s = ctx->stream;
  const long n = ctx->nU;
  double* tmp = ctx->Ustages[2];
  double* Yk = ctx->Ybar;
  int rc = fe_transpose(ctx, 2, U2, Ybar, tmp, dt, &si[2]);
  if (rc) return rc;
  HIPC(launch_axpby(n, 2.0 / 3.0, tmp, 0.0, Yk, s));       // Y2
  HIPC(launch_axpby(n, 0.75, Yk, 1.0 / 3.0, Ybar, s));     // Ubar = 1/3 Y3 + 3/4 Y2
  rc = fe_transpose(ctx, 1, U1, Yk, tmp, dt, &si[1]);
  if (rc) return rc;
  HIPC(launch_axpby(n, 0.25, tmp, 0.0, Yk, s));            // Y1
  rc = fe_transpose(ctx, 0, Un, Yk, tmp, dt, &si[0]);
  if (rc) return rc;
  HIPC(launch_axpby(n, 1.0, tmp, 1.0, Ybar, s));           // Ubar += J_FE(Un)^T Y1
  return DFDG_OK;
}

// Cotangent of E = 1/2 U . U (orthonormal broken basis: the kinetic energy of the state).
extern "C" int dfdg_energy_vjp(dfdg_ctx* ctx, const double* U, double Ebar, double* Ubar) {
  NEED_BOUND(ctx);
  if (!U || !Ubar) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (!std::isfinite(Ebar)) return fail(ctx, DFDG_E_INVALID_ARG, "Ebar must be finite");
  HIPC(launch_axpby(ctx->nU, Ebar, U, 0.0, Ubar, ctx->stream));
  return DFDG_OK;
}

static int vjp_info(dfdg_ctx* ctx, const dfdg_solve_info (&si)[3], const dfdg_solve_info* fw, int nfw,
                    dfdg_step_info* info) {
  dfdg_step_info st{};
  st.status = DFDG_OK;
  for (int i = 0; i < 3; ++i) {
    st.iterations[i] = si[i].iterations;
    st.max_rel_residual = std::max(st.max_rel_residual, si[i].rel_residual);
    if (si[i].status != DFDG_OK) st.status = si[i].status;
  }
  for (int i = 0; i < nfw; ++i)
    if (fw[i].status != DFDG_OK) st.status = fw[i].status;
  if (info) *info = st;
  if (st.status != DFDG_OK) return fail(ctx, st.status, "a facet solve of the adjoint step did not converge");
  return DFDG_OK;
}

extern "C" int dfdg_rk3_step_vjp(dfdg_ctx* ctx, const double* Un, double* Ybar, double dt, dfdg_step_info* info) {
  NEED_BOUND(ctx);
  if (!Un || !Ybar) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, DFDG_E_INVALID_ARG, "dt must be finite and > 0");
  if (ctx->prm.precision != DFDG_FP64) return fail(ctx, DFDG_E_UNSUPPORTED, "the adjoint runs in FP64 only");
  use_integrator(ctx, 1);
  double* U1 = ctx->Ustages[0];
  double* U2 = ctx->Ustages[1];
  dfdg_solve_info fw[2]{}, si[3]{};
  int rc = rk_stage(ctx, 0, Un, Un, 0.0, 1.0, dt, U1, &fw[0]);
  if (!rc) rc = rk_stage(ctx, 1, U1, Un, 0.75, 0.25, dt, U2, &fw[1]);
  if (rc) return rc;
  rc = rk3_vjp_core(ctx, Un, U1, U2, Ybar, dt, si);
  if (rc) return rc;
  return vjp_info(ctx, si, fw, 2, info);
}

extern "C" int dfdg_rk3_step_vjp_stages(dfdg_ctx* ctx, const double* Un, const double* U1, const double* U2,
                                        double* Ybar, double dt, dfdg_step_info* info) {
  NEED_BOUND(ctx);
  if (!Un || !U1 || !U2 || !Ybar) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (Ybar == Un || Ybar == U1 || Ybar == U2) return fail(ctx, DFDG_E_INVALID_ARG, "Ybar must not alias a state");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, DFDG_E_INVALID_ARG, "dt must be finite and > 0");
  if (ctx->prm.precision != DFDG_FP64) return fail(ctx, DFDG_E_UNSUPPORTED, "the adjoint runs in FP64 only");
  dfdg_solve_info si[3]{};
  int rc = rk3_vjp_core(ctx, Un, U1, U2, Ybar, dt, si);
  if (rc) return rc;
  return vjp_info(ctx, si, nullptr, 0, info);
}

// ---------------------------------------------------------------------------------------
// diagnostics, evaluation, measurement
// ---------------------------------------------------------------------------------------
extern "C" int dfdg_diagnostics(dfdg_ctx* ctx, const double* U, dfdg_diag* out) {
  NEED_BOUND(ctx);
  if (!U || !out) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  HIPC(el_diagnostics(ctx, U, ctx->partials, ctx->diagres, ctx->stream));
  double res[4];
  HIPC(hipMemcpyAsync(ctx->pinned, ctx->diagres, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));
  std::memcpy(res, ctx->pinned, sizeof(res));
  out->energy = res[0];
  out->enstrophy = res[1];
  out->max_div = res[2];
  out->max_normal_jump = res[3];
  return DFDG_OK;
}

extern "C" int dfdg_diagnostics_noalloc(dfdg_ctx* ctx, const double* U, dfdg_diag* out) {
  NEED_BOUND(ctx);
  if (!U || !out) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (diag_blocks(ctx->T) > kNoAllocDiagBlocks)
    return fail(ctx, DFDG_E_INVALID_ARG,
                "dfdg_diagnostics_noalloc: " + std::to_string(ctx->T) + " elements exceed its static scratch (at most " +
                    std::to_string(kNoAllocDiagBlocks * 128) + ")");
  int dev = -1;
  HIPC(hipGetDevice(&dev));
  double* part = nullptr;
  HIPC(noalloc_scratch(&part));  // the same address as at set-up when called on that device
  if (part != ctx->noalloc)
    return fail(ctx, DFDG_E_INVALID_ARG, "dfdg_diagnostics_noalloc: called with another device current (" +
                                             std::to_string(dev) + ") than at set-up");
  double* res = part + 4 * kNoAllocDiagBlocks;
  // every partial and result is written before it is read: nothing to clear
  HIPC(el_diagnostics(ctx, U, part, res, ctx->stream));
  double r[4];
  HIPC(hipMemcpyAsync(ctx->pinned, res, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));
  std::memcpy(r, ctx->pinned, sizeof(r));
  out->energy = r[0];
  out->enstrophy = r[1];
  out->max_div = r[2];
  out->max_normal_jump = r[3];
  return DFDG_OK;
}

extern "C" int dfdg_eval(dfdg_ctx* ctx, const double* U, int npts, const double* ref, double* out) {
  NEED_BOUND(ctx);
  if (!U || !ref || !out) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (npts < 1 || npts > kMaxEvalPts) return fail(ctx, DFDG_E_INVALID_ARG, "npts must be in 1..1024");
  const int P = ctx->P;
  std::vector<double> tab((size_t)npts * P);
  for (int p = 0; p < npts; ++p) {
    if (ctx->dim == 3) dubiner3(ctx->K, ref[3 * p], ref[3 * p + 1], ref[3 * p + 2], &tab[(size_t)p * P], nullptr);
    else dubiner(ctx->K, ref[2 * p], ref[2 * p + 1], &tab[(size_t)p * P], nullptr);
  }
  HIPC(hipMemcpyAsync(ctx->evaltab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  if (ctx->dim == 3) HIPC(launch_eval3(ctx->K, npts, ctx->g, ctx->evaltab, U, out, ctx->stream));
  else HIPC(launch_eval(ctx->K, npts, ctx->g, ctx->evaltab, U, out, ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));  // tab is a host temporary
  return DFDG_OK;
}

extern "C" int dfdg_debug_facet_rhs(dfdg_ctx* ctx, double* g) {
  NEED_BOUND(ctx);
  if (!g) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  HIPC(hipMemcpyAsync(g, ctx->gv, ctx->nL * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));
  return DFDG_OK;
}

extern "C" int dfdg_debug_vcycle(dfdg_ctx* ctx, const double* b, double* z) {
  NEED_BOUND(ctx);
  if (!b || !z) return fail(ctx, DFDG_E_INVALID_ARG, "null pointer");
  if (ctx->prm.precond != DFDG_AMG) return fail(ctx, DFDG_E_INVALID_ARG, "V-cycle needs an AMG context");
  hipStream_t s = ctx->stream;
  const long NF = ctx->NF;
  const PcgBufs& pb = ctx->pbt;
  PcgScalars st{};  // a running state whose stopping test never fires
  st.rz = 1.0; st.rr = 1.0; st.gg = 1.0; st.tol2 = -1.0; st.maxit = 1 << 30; st.it = 2;
  HIPC(hipMemcpyAsync(pb.sc, &st, sizeof(st), hipMemcpyHostToDevice, s));
  const long G = ctx->g.fgrid;
  HIPC(launch_fill(2 * G, 1.0, pb.rz[0], s));
  HIPC(hipMemcpyAsync(ctx->r, b, ctx->nL * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (ctx->prm.mg_fp32) HIPC((launch_vcycle<float, double>(NF, ctx->g, ctx->A, ctx->mg, ctx->r, ctx->z, pb.rz[0], pb.sc, s)));
  else HIPC((launch_vcycle<double, double>(NF, ctx->g, ctx->A, ctx->mg, ctx->r, ctx->z, pb.rz[0], pb.sc, s)));
  HIPC(hipMemcpyAsync(z, ctx->z, ctx->nL * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPC(hipStreamSynchronize(s));
  return DFDG_OK;
}

extern "C" int dfdg_time_kernel(dfdg_ctx* ctx, int which, int reps, float* ms, double* bytes) {
  NEED_BOUND(ctx);
  if (!ms || reps < 1) return fail(ctx, DFDG_E_INVALID_ARG, "bad arguments");
  if (which == 3 && ctx->prm.precision != DFDG_MIXED) return fail(ctx, DFDG_E_INVALID_ARG, "FP32 SpMV needs a MIXED context");
  if (which == 4 && ctx->prm.precond != DFDG_AMG) return fail(ctx, DFDG_E_INVALID_ARG, "V-cycle needs an AMG context");
  if (which < 0 || which > 6) return fail(ctx, DFDG_E_INVALID_ARG, "unknown kernel id");
  hipStream_t s = ctx->stream;
  const long T = ctx->T, E = ctx->E, NF = ctx->NF, P = ctx->P, NS = ctx->A.ns;
  // a running PCG state whose stopping test never fires, and finite partials
  const PcgBufs& pb = ctx->pbt;
  PcgScalars st{};
  st.rz = 1.0; st.rr = 1.0; st.gg = 1.0; st.tol2 = -1.0; st.maxit = 1 << 30; st.it = 2;
  HIPC(hipMemcpyAsync(pb.sc, &st, sizeof(st), hipMemcpyHostToDevice, s));
  const long G = ctx->g.fgrid;
  HIPC(launch_fill(2 * G, 1.0, pb.rz[0], s));
  HIPC(launch_fill(2 * G, 1.0, pb.rz[1], s));
  HIPC(launch_fill(2 * G, 1.0, pb.pq, s));
  auto launch = [&]() -> hipError_t {
    switch (which) {
      case 0: return launch_pcg_spmv(NF, ctx->g, ctx->A, ctx->z, ctx->p[0], ctx->p[1], ctx->Sp, pb, 2, s);
      case 1: return launch_pcg_update(NF, ctx->prm.precond == DFDG_BLOCK_JACOBI ? 1 : 0, ctx->g, ctx->A, ctx->p[1], ctx->Sp,
                                       ctx->gv, ctx->r, ctx->z, pb, 1, s);  // writes rz[1], reads rz[0]
      case 2: return el_residual(ctx, false, ctx->Ustage, ctx->Lbuf, s);
      case 5: return el_cond_rhs(ctx, false, ctx->Lbuf, s);
      case 6:  // the stage epilogue u = a U^n + b (U^s + dt W(F - C^T lambda)), in place
        return el_recover(ctx, false, ctx->Lbuf, ctx->lamx, ctx->Ustage, 1, 0.5, ctx->Ustage, 0.5, ctx->Ustage, 1e-30,
                          s);
      case 4:
        if (ctx->prm.mg_fp32) return launch_vcycle<float, double>(NF, ctx->g, ctx->A, ctx->mg, ctx->r, ctx->z, pb.rz[0], pb.sc, s);
        return launch_vcycle<double, double>(NF, ctx->g, ctx->A, ctx->mg, ctx->r, ctx->z, pb.rz[0], pb.sc, s);
      default: return launch_pcg32_spmv(NF, ctx->g, ctx->A, ctx->z32, ctx->p32[0], ctx->p32[1], ctx->Sp32, pb, 2, s);
    }
  };
  HIPC(launch());  // warm-up
  // single-kernel measurements (SpMV, residual) attach the events to the dispatch itself,
  // so that end - start is the kernel's execution; the V-cycle (several kernels) is
  // bracketed by events recorded on the stream
  // (the tetrahedral condensation kernels do not take dispatch events)
  const bool single = which == 0 || which == 2 || which == 3 || ((which == 5 || which == 6) && ctx->dim == 2);
  std::vector<hipEvent_t> ev(2 * (size_t)reps);
  for (auto& e : ev) HIPC(hipEventCreate(&e));
  for (int i = 0; i < reps; ++i) {
    if (single) {
      set_dispatch_events(ev[2 * i], ev[2 * i + 1]);
      hipError_t e = launch();
      set_dispatch_events(nullptr, nullptr);
      HIPC(e);
    } else {
      HIPC(hipEventRecord(ev[2 * i], s));
      HIPC(launch());
      HIPC(hipEventRecord(ev[2 * i + 1], s));
    }
  }
  HIPC(hipEventSynchronize(ev.back()));
  double tot = 0;
  for (int i = 0; i < reps; ++i) {
    float t = 0;
    HIPC(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
    tot += t;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  *ms = (float)(tot / reps);
  if (bytes) {
    double b = 0;
    switch (which) {
      case 0:
        if (ctx->A.mfq)  // element pass: Jinv, (D D^T)^{-1}, per face id, code, sqrt(|F|/det), normal,
                         // z and p_old gathered, contributions out; face pass: 2 offsets, both
                         // contributions, z, p_old in, p_new, Sp out
          b = T * (9 * 8.0 + nGpk3(ctx->K) * 8.0 + 4 * (2 * 4.0 + 4 * 8.0) + 4 * NF * 2 * 8.0 + 4 * NF * 8.0) +
              E * (2 * 4.0 + 6.0 * NF * 8.0);
        else
          b = E * (NS * NF * NF * 8.0 + NS * 4.0 + 4.0 * NF * 8.0);  // S, cols, z, p_old, p_new, Sp
        break;
      case 1: b = E * NF * 8.0 * 8.0; break;                                                  // p, Sp, x, r, M^{-1} in; x, r, z out
      case 2:  // U (own + neighbours) in, L out, Jinv + 1/sqrt(detJ); per facet nbr, code, normal,
               // |F| (and sigma if nu != 0)
        if (ctx->dim == 3)
          b = T * (2.0 * 3 * P * 8.0 + 10 * 8.0 + 4 * (2 * 4.0 + (ctx->prm.nu != 0.0 ? 5 : 4) * 8.0));
        else
          b = T * (2.0 * 2 * P * 8.0 + 5 * 8.0 + 3 * (2 * 4.0 + (ctx->prm.nu != 0.0 ? 4 : 3) * 8.0));
        break;
      case 4: {
        // finest level: 4 BSR sweeps + 17 vector passes; transfers and coarse levels:
        // every CSR entry (value and 4-byte column) once per use, vectors once.  Values
        // and vectors in the cycle's precision (8 or 4 bytes; finest-level S in 2 bytes
        // when it is stored in FP16).
        const double vb = ctx->prm.mg_fp32 ? 4.0 : 8.0;
        const double sv = ctx->A.vals16 ? 4.0 * nPairs(NF, NS) / (NS * NF * NF) : vb;
        const double sbytes = E * (NS * NF * NF * sv + NS * 4.0);
        b = 4 * sbytes + 17.0 * E * NF * vb;
        const AmgHierarchy& H = ctx->H;
        for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
          const AmgLevel& L = H.lv[l];
          const double nn = H.lv[l + 1].A.n;
          if (l == 0) {  // transfers of the finest level
            b += (L.P.nnz() + L.R.nnz()) * (vb + 4.0) + (2.0 * L.A.n + 2.0 * nn) * vb;
          } else {  // restriction with the smoothing step, prolongation with the post-smoothing
            b += (L.A.nnz() + L.R.nnz() + L.RA.nnz() + L.AP.nnz() + L.P.nnz()) * (vb + 4.0) +
                 5.0 * L.A.n * vb + 2.0 * nn * vb;
          }
        }
        b += H.n_coarse * (double)H.n_coarse * vb;
        break;
      }
      case 5:    // F in, face coefficients out; Jinv; the packed local inverse (FE4: and det J,
      case 6: {  // 1/sqrt(det J)); per face code, sqrt(|F|/det), normal (6: face id and the
                 // face's multipliers in, and the stage state U in and out, as timed here)
        const int dm = ctx->dim, nfac = dm + 1;
        const double loc = ctx->g.G4 ? nG4pk(ctx->K) * 8.0 + 16.0 : (dm == 3 ? nGpk3(ctx->K) : nGpk(ctx->K)) * 8.0;
        const double per_face = which == 5 ? 4.0 + (1 + dm) * 8.0 + NF * 8.0 : 2 * 4.0 + (1 + dm) * 8.0 + NF * 8.0;
        b = T * (dm * P * 8.0 + dm * dm * 8.0 + loc + nfac * per_face + (which == 6 ? 2.0 * dm * P * 8.0 : 0.0));
        break;
      }
      default: b = E * (NS * NF * NF * 4.0 + NS * 4.0 + 4.0 * NF * 4.0); break;
    }
    *bytes = b;
  }
  return DFDG_OK;
}

// ---------------------------------------------------------------------------------------
// host inspection
// ---------------------------------------------------------------------------------------
extern "C" int dfdg_debug_basis(int k, int npts, const double* pts, double* vals, double* grads) {
  if (k < 1 || k > kMaxK || npts < 1 || !pts || !vals) return DFDG_E_INVALID_ARG;
  const int P = nP(k);
  std::vector<double> g(2 * P);
  for (int p = 0; p < npts; ++p) {
    dubiner(k, pts[2 * p], pts[2 * p + 1], vals + (size_t)p * P, g.data());
    if (grads) std::memcpy(grads + (size_t)p * 2 * P, g.data(), 2 * P * sizeof(double));
  }
  return DFDG_OK;
}

extern "C" int dfdg_debug_residual_rule(int k, int* npts, double* pts, double* w) {
  if (k < 1 || k > kMaxK || !npts) return DFDG_E_INVALID_ARG;
  std::vector<double> q, qw;
  residual_volume_rule(k, q, qw);
  *npts = (int)qw.size();
  if (pts) std::memcpy(pts, q.data(), q.size() * sizeof(double));
  if (w) std::memcpy(w, qw.data(), qw.size() * sizeof(double));
  return DFDG_OK;
}

extern "C" int dfdg_debug_basis3(int k, int npts, const double* pts, double* vals, double* grads) {
  if (k < 1 || k > kMaxK3 || npts < 1 || !pts || !vals) return DFDG_E_INVALID_ARG;
  const int P = nP3(k);
  std::vector<double> g(3 * P);
  for (int p = 0; p < npts; ++p) {
    dubiner3(k, pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], vals + (size_t)p * P, g.data());
    if (grads) std::memcpy(grads + (size_t)p * 3 * P, g.data(), 3 * P * sizeof(double));
  }
  return DFDG_OK;
}

extern "C" int dfdg_debug_rule3(int k, int which, int* npts, double* pts, double* w) {
  if (k < 1 || k > kMaxK3 || !npts || which < 0 || which > 2) return DFDG_E_INVALID_ARG;
  RefTables t;
  build_ref_tables3(k, t);
  const std::vector<double>& q = which == 0 ? t.vq : which == 1 ? t.fs : t.pq;
  const std::vector<double>& qw = which == 0 ? t.vw : which == 1 ? t.fw : t.pw;
  *npts = (int)qw.size();
  if (pts) std::memcpy(pts, q.data(), q.size() * sizeof(double));
  if (w) std::memcpy(w, qw.data(), qw.size() * sizeof(double));
  return DFDG_OK;
}

extern "C" int dfdg_debug_facet_matrix(const dfdg_ctx* ctx, int32_t* cols, double* vals) {
  if (!ctx || !cols || !vals) return DFDG_E_INVALID_ARG;
  std::memcpy(cols, ctx->hs.cols.data(), ctx->hs.cols.size() * sizeof(int32_t));
  std::memcpy(vals, ctx->hs.vals.data(), ctx->hs.vals.size() * sizeof(double));
  return DFDG_OK;
}

extern "C" int dfdg_debug_multigrid_matrix(const dfdg_ctx* ctx, int level, int which, int64_t* n_rows,
                                           int64_t* n_cols, int64_t* nnz, int64_t* ptr, int32_t* cols,
                                           double* vals) {
  if (!ctx || !n_rows || !n_cols || !nnz) return DFDG_E_INVALID_ARG;
  const int L = (int)ctx->H.lv.size();
  if (level < 0 || level >= L || which < 0 || which > 4) return DFDG_E_INVALID_ARG;
  if (which == 2) {  // dense coarsest pseudo-inverse, as a full CSR
    if (level != L - 1) return DFDG_E_INVALID_ARG;
    const long n = ctx->H.n_coarse;
    *n_rows = *n_cols = n;
    *nnz = n * n;
    if (ptr && cols && vals) {
      for (long i = 0; i <= n; ++i) ptr[i] = i * n;
      for (long i = 0; i < n * n; ++i) {
        cols[i] = (int32_t)(i % n);
        vals[i] = ctx->H.coarse_inv[i];
      }
    }
    return DFDG_OK;
  }
  const AmgLevel& lv = ctx->H.lv[level];
  const Csr& M = which == 0 ? lv.A : which == 1 ? lv.P : which == 3 ? lv.AP : lv.RA;
  if (which != 0 && level == L - 1) return DFDG_E_INVALID_ARG;
  if (which >= 3 && M.n == 0) return DFDG_E_INVALID_ARG;
  *n_rows = M.n;
  *n_cols = M.m;
  *nnz = M.nnz();
  if (ptr && cols && vals) {
    for (int i = 0; i <= M.n; ++i) ptr[i] = M.ptr[i];
    for (long k = 0; k < M.nnz(); ++k) {
      cols[k] = M.col[k];
      vals[k] = M.val[k];
    }
  }
  return DFDG_OK;
}

extern "C" int dfdg_debug_multigrid(const dfdg_ctx* ctx, int max_levels, int* n_levels, int64_t* rows,
                                    int64_t* nnz, double* rho) {
  if (!ctx || !n_levels || max_levels < 0 || (max_levels > 0 && (!rows || !nnz || !rho))) return DFDG_E_INVALID_ARG;
  const int L = (int)ctx->H.lv.size();
  *n_levels = L;
  for (int l = 0; l < std::min(L, max_levels); ++l) {
    rows[l] = ctx->H.lv[l].A.n;
    nnz[l] = ctx->H.lv[l].A.nnz();
    rho[l] = ctx->H.lv[l].lmax;
  }
  return DFDG_OK;
}
