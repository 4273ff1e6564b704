// C ABI of the ddhelm library: set-up of the partition and coarse factors, the
// batched Schwarz preconditioner and the outer FGMRES driver (host side).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "ddhelm.h"
#include "coarse.hpp"
#include "gcoarse.hpp"
#include "kernels.hpp"
#include "net_host.hpp"
#include "outer.hpp"
#include "stencil.hpp"

using ddh::cplx;
using ddh::SubDesc;

namespace {

thread_local std::string g_last_error;

dd_status fail(dd_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define DD_HIP(expr)                                                                                       \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess)                                                                                   \
      return fail(e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP,                                          \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                                       \
  } while (0)

#define DD_TRY(expr)                  \
  do {                                \
    dd_status s_ = (expr);            \
    if (s_ != DD_OK) return s_;       \
  } while (0)

// A factorisation whose smallest |pivot| is below this fraction of the largest |entry| of
// the factored matrix is reported as singular: at that ratio the matrix is within rounding
// of singular in FP64 (a pivot perturbed at 1e-16 relative changes the solve at ~1e-4), as
// when k^2 meets an eigenvalue of a local or coarse pencil.
constexpr double kTinyPivot = 1e-12;

dd_status check_pivots(const std::string& what, double min_pivot, double max_entry) {
  if (!(min_pivot > 0.0) || !std::isfinite(min_pivot) || !(max_entry > 0.0) || !std::isfinite(max_entry))
    return fail(DD_ESINGULAR, what + " is singular (zero or non-finite pivot)");
  const double ratio = min_pivot / max_entry;
  if (ratio < kTinyPivot) {
    char b[160];
    std::snprintf(b, sizeof(b), " is singular to working precision: min |pivot| / max |entry| = %.3e < %.0e",
                  ratio, kTinyPivot);
    return fail(DD_ESINGULAR, what + b);
  }
  return DD_OK;
}

constexpr int kOuterBlocks = 1024;   // workgroups of the grid-stride outer kernels
constexpr int kMaxRestart = 4000;    // Givens kernel stages a restart cycle in LDS
constexpr int kMaxGraphSteps = 64;   // outer steps per captured graph
constexpr int kEvPerStep = 8;        // phase events recorded per outer step

}  // namespace

namespace ddh {
dd_status fail_msg(dd_status s, const std::string& msg) { return fail(s, msg); }
}  // namespace ddh

struct dd_handle {
  dd_params p{};
  int n = 0;
  long long ndof = 0;
  int nsub = 0, nrhs = 1, prec = 64, maxit = 0, restart = 0;
  std::vector<int> cuts_x, cuts_y;
  std::vector<SubDesc> subs_h;
  long long nfine = 0, ncoarse = 0, nfac = 0;
  int max_nj = 0, max_nc = 0;
  ddh::Consts cs{};
  std::vector<double> pivmin_h;
  // device
  SubDesc* subs = nullptr;
  int* order = nullptr;
  cplx<double>* Ec = nullptr;
  cplx<double>* fac = nullptr;
  double* pivmin = nullptr;
  void* F = nullptr;
  void* W = nullptr;
  void* X = nullptr;
  void* U = nullptr;
  void* V = nullptr;
  cplx<double>* R = nullptr;
  cplx<double>* Sc = nullptr;   // coarse vectors kept by each subdomain solve for its recovery
  int* iters = nullptr;
  int* flags = nullptr;
  unsigned long long* counters = nullptr;
  // outer FGMRES
  cplx<double>* Vo = nullptr;   // [nrhs][restart + 1][ndof]
  cplx<double>* Zo = nullptr;   // [nrhs][restart][ndof]
  cplx<double>* part = nullptr; // [nrhs][pstride][chunks] (launch_dots), [nrhs][chunks][pstride] + segments (dots2)
  cplx<double>* coef = nullptr; // [nrhs][pstride]
  cplx<double>* ca = nullptr;   // [nrhs][restart] delayed-CGS2 update coefficients
  cplx<double>* cb = nullptr;
  cplx<double>* scal = nullptr; // [nrhs][4]
  int pstride = 0;
  ddh::OuterState os{};
  int* done_h = nullptr;        // pinned
  double* res_h = nullptr;      // pinned
  hipEvent_t ev[8] = {};        // phase timers of dd_solve
  bool ev_ok = false;
  int* jdev = nullptr;          // device-side outer step index
  // launch configuration (dd_autotune)
  int inner_nt = ddh::kInnerThreads;
  bool lpt = true;              // subdomain solves launched largest tile first
  int dots_blocks = 0;          // grid of the outer dot sweep (0 = default)
  std::vector<hipEvent_t> sev;  // per-step phase events, kEvPerStep per step slot
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  dd_net* net = nullptr;        // attached guess network (borrowed)
  // exact local solves (local_solver == DD_LOCAL_DIRECT)
  bool direct = false;
  cplx<double>* ffac = nullptr; // twisted block factors of the local matrices
  long long* foff = nullptr;    // [nsub] factor offsets
  std::vector<long long> foff_h;
  long long nffac = 0;
  // two-level method (coarse_intervals > 0)
  ddh::GlobalCoarse* gc = nullptr;
  // multi-launch subdomain solves (inner_launch == DD_INNER_MULTI)
  bool multi = false;
  ddh::MultiArgs mk{};          // workspaces; per call the caller's vectors are filled in
  int* active_h = nullptr;      // pinned

  std::vector<void*> allocs;

  template <typename T>
  dd_status alloc(T** ptr, size_t count) {
    void* q = nullptr;
    DD_HIP(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)));
    allocs.push_back(q);
    *ptr = (T*)q;
    return DD_OK;
  }
  void release() {
    delete gc;
    gc = nullptr;
    for (void* q : allocs) (void)hipFree(q);
    allocs.clear();
    if (ev_ok)
      for (int e = 0; e < 8; ++e) (void)hipEventDestroy(ev[e]);
    ev_ok = false;
    for (hipEvent_t e : sev) (void)hipEventDestroy(e);
    sev.clear();
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    graph_exec = nullptr;
    graph = nullptr;
    cap_stream = nullptr;
    if (active_h) (void)hipHostFree(active_h);
    active_h = nullptr;
    if (done_h) (void)hipHostFree(done_h);
    if (res_h) (void)hipHostFree(res_h);
    done_h = nullptr;
    res_h = nullptr;
  }
};

extern "C" {

void dd_default_params(dd_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->k = 20.0;
  p->ppwl = 10.0;
  p->n_intervals = 0;
  p->px = p->py = 2;
  p->overlap = 1;
  p->local_bc = DD_LOCAL_IMPEDANCE;
  p->deflation = DD_DEFLATION_LINEAR;
  p->inner_precision = 64;
  p->inner_tol = 1e-2;
  p->inner_maxit = 100;
  p->outer_tol = 1e-6;
  p->outer_maxit = 3000;   /* also the restart length unless outer_restart > 0 */
  p->outer_restart = 0;
  p->nrhs = 1;
  p->use_graph = 1;
  p->graph_steps = 8;
}

const char* dd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

dd_status validate_and_plan(const dd_params* p, dd_handle* h) {
  if (!(p->k > 0.0) || !std::isfinite(p->k)) return fail(DD_EINVAL, "k must be positive and finite");
  int n = p->n_intervals;
  if (n <= 0) {
    if (!(p->ppwl > 0.0)) return fail(DD_EINVAL, "ppwl must be positive when n_intervals <= 0");
    n = (int)std::ceil(p->k * p->ppwl / (2.0 * M_PI) - 1e-9);
  }
  if (n < 4 || n > 65536) return fail(DD_EINVAL, "N must be in [4, 65536]");
  if (p->px < 1 || p->py < 1 || p->px > n || p->py > n) return fail(DD_EINVAL, "bad subdomain counts");
  if (p->overlap < 1) return fail(DD_EINVAL, "overlap must be at least one element layer");
  if (p->local_bc != DD_LOCAL_IMPEDANCE && p->local_bc != DD_LOCAL_DIRICHLET)
    return fail(DD_EINVAL, "local_bc must be DD_LOCAL_IMPEDANCE or DD_LOCAL_DIRICHLET");
  if (p->deflation != DD_DEFLATION_LINEAR && p->deflation != DD_DEFLATION_BEZIER)
    return fail(DD_EINVAL, "deflation must be DD_DEFLATION_LINEAR or DD_DEFLATION_BEZIER");
  if (p->inner_precision != 64 && p->inner_precision != 32) return fail(DD_EINVAL, "inner_precision must be 64 or 32");
  if (p->local_solver != DD_LOCAL_DEFLATED_GMRES && p->local_solver != DD_LOCAL_DIRECT)
    return fail(DD_EINVAL, "local_solver must be DD_LOCAL_DEFLATED_GMRES or DD_LOCAL_DIRECT");
  if (p->local_solver == DD_LOCAL_DIRECT && p->inner_precision != 64)
    return fail(DD_EINVAL, "direct local solves are FP64: inner_precision must be 64");
  if (!(p->inner_tol > 0.0 && p->inner_tol < 1.0)) return fail(DD_EINVAL, "inner_tol must be in (0, 1)");
  if (p->inner_maxit < 1 || p->inner_maxit > 1000) return fail(DD_EINVAL, "inner_maxit must be in [1, 1000]");
  if (!(p->outer_tol > 0.0 && p->outer_tol < 1.0)) return fail(DD_EINVAL, "outer_tol must be in (0, 1)");
  if (p->outer_maxit < 1) return fail(DD_EINVAL, "outer_maxit must be >= 1");
  if (p->nrhs < 1 || p->nrhs > 64) return fail(DD_EINVAL, "nrhs must be in [1, 64]");
  if (p->coarse_intervals != 0 &&
      (p->coarse_intervals < 2 || p->coarse_intervals > n || p->coarse_intervals - 1 > ddh::kMaxGlobalCoarse))
    return fail(DD_EINVAL, "coarse_intervals must be 0 (one-level) or in [2, N] with at most 1025 intervals");
  if (p->use_graph && (p->graph_steps < 1 || p->graph_steps > kMaxGraphSteps))
    return fail(DD_EINVAL, "graph_steps must be in [1, 64]");
  if (p->inner_launch != DD_INNER_FUSED && p->inner_launch != DD_INNER_MULTI)
    return fail(DD_EINVAL, "inner_launch must be DD_INNER_FUSED or DD_INNER_MULTI");
  if (p->inner_launch == DD_INNER_MULTI) {
    if (p->local_solver != DD_LOCAL_DEFLATED_GMRES)
      return fail(DD_EINVAL, "the multi-launch form runs deflated-GMRES local solves");
    if (p->inner_precision != 64) return fail(DD_EINVAL, "the multi-launch form needs inner_precision 64");
    if (p->nrhs != 1) return fail(DD_EINVAL, "the multi-launch form needs nrhs 1");
    if (p->use_graph) return fail(DD_EINVAL, "the multi-launch form needs use_graph 0");
    if (p->inner_maxit > ddh::kMultiMaxIt) return fail(DD_EINVAL, "the multi-launch form needs inner_maxit <= 256");
  }
  auto cuts = [&](const int* c, int parts, std::vector<int>& out) -> dd_status {
    out.resize(parts + 1);
    for (int q = 0; q <= parts; ++q) out[q] = c ? c[q] : (int)(((long long)q * n) / parts);
    if (out[0] != 0 || out[parts] != n) return fail(DD_EINVAL, "cut points must start at 0 and end at N");
    for (int q = 0; q < parts; ++q)
      if (out[q + 1] - out[q] < 1) return fail(DD_EINVAL, "cut points must be strictly increasing");
    return DD_OK;
  };
  DD_TRY(cuts(p->cuts_x, p->px, h->cuts_x));
  DD_TRY(cuts(p->cuts_y, p->py, h->cuts_y));
  h->p = *p;
  h->p.cuts_x = nullptr;
  h->p.cuts_y = nullptr;
  h->n = n;
  h->ndof = (long long)(n - 1) * (n - 1);
  h->nsub = p->px * p->py;
  h->nrhs = p->nrhs;
  h->prec = p->inner_precision;
  h->maxit = p->inner_maxit;
  h->restart = p->outer_restart > 0 ? std::min(p->outer_restart, p->outer_maxit) : p->outer_maxit;
  if (h->restart > kMaxRestart)
    return fail(DD_EINVAL, "outer restart length (outer_maxit when outer_restart <= 0) must be <= 4000");
  const int ov = p->overlap;
  const bool imp = p->local_bc == DD_LOCAL_IMPEDANCE;
  h->subs_h.clear();
  h->direct = p->local_solver == DD_LOCAL_DIRECT;
  h->multi = p->inner_launch == DD_INNER_MULTI;
  h->foff_h.clear();
  long long off = 0, coff = 0, goff = 0, foff = 0;
  for (int qy = 0; qy < p->py; ++qy) {
    for (int qx = 0; qx < p->px; ++qx) {
      SubDesc d{};
      d.ax = std::max(0, h->cuts_x[qx] - ov);
      d.bx = std::min(n, h->cuts_x[qx + 1] + ov);
      d.ay = std::max(0, h->cuts_y[qy] - ov);
      d.by = std::min(n, h->cuts_y[qy + 1] + ov);
      int i0, i1, j0, j1;
      if (imp) {
        i0 = std::max(d.ax, 1); i1 = std::min(d.bx, n - 1);
        j0 = std::max(d.ay, 1); j1 = std::min(d.by, n - 1);
      } else {
        i0 = d.ax + 1; i1 = d.bx - 1; j0 = d.ay + 1; j1 = d.by - 1;
      }
      d.i0 = i0; d.j0 = j0; d.nx = i1 - i0 + 1; d.ny = j1 - j0 + 1;
      if (d.nx < 2 || d.ny < 2) return fail(DD_EINVAL, "every subdomain needs at least 2 x 2 local unknowns");
      d.oi0 = std::max(h->cuts_x[qx], 1); d.oi1 = h->cuts_x[qx + 1] - 1;
      d.oj0 = std::max(h->cuts_y[qy], 1); d.oj1 = h->cuts_y[qy + 1] - 1;
      d.mx = d.nx / 2; d.my = d.ny / 2;
      d.defl = p->deflation;
      if (d.defl == DD_DEFLATION_LINEAR) {
        d.bmx = d.mx; d.bmy = d.my;
      } else {
        d.bmx = 2 * d.mx; d.bmy = (d.my + 1) / 2;
      }
      d.ncp = d.bmx * d.bmy;
      if (d.bmx > ddh::kMaxMx)
        return fail(DD_EINVAL, "subdomain too wide for the coarse kernels (coarse block size > 128)");
      if (h->direct) {
        if (d.nx > ddh::kMaxMx) return fail(DD_EINVAL, "subdomain too wide for direct local solves (nx > 128)");
        h->foff_h.push_back(foff);
        foff += ddh::coarse_factor_size(d.nx, d.ny);
      }
      d.robin = 0;
      if (imp) d.robin = (d.ax > 0 ? 1 : 0) | (d.bx < n ? 2 : 0) | (d.ay > 0 ? 4 : 0) | (d.by < n ? 8 : 0);
      d.off = off; d.coff = coff; d.goff = goff;
      off += (long long)d.nx * d.ny;
      coff += (long long)d.mx * d.my;
      goff += d.defl == DD_DEFLATION_LINEAR ? ddh::coarse_factor_size(d.mx, d.my)
                                            : ddh::coarse_factor_size_paired(d.bmx, d.bmy);
      h->max_nj = std::max(h->max_nj, d.nx * d.ny);
      h->max_nc = std::max(h->max_nc, d.ncp);
      h->subs_h.push_back(d);
    }
  }
  h->nfine = off;
  h->ncoarse = coff;
  h->nfac = goff;
  h->nffac = foff;
  h->cs.n = n;
  h->cs.nsub = h->nsub;
  h->cs.k = p->k;
  h->cs.h = 1.0 / n;
  h->cs.kh = p->k / n;
  h->cs.kh2 = h->cs.kh * h->cs.kh;
  return DD_OK;
}

template <typename T>
dd_status check_lds(dd_handle* h) {
  int dev = 0, maxlds = 0;
  DD_HIP(hipGetDevice(&dev));
  DD_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  size_t need = h->direct ? ddh::direct_lds_bytes(h->max_nj) : ddh::inner_lds_bytes<T>(h->max_nj, h->max_nc, h->maxit);
  if (need > (size_t)maxlds)
    return fail(DD_EINVAL, "subdomain tile too large for LDS (" + std::to_string(need) + " > " +
                               std::to_string(maxlds) + " bytes); use more subdomains or fewer inner iterations");
  return DD_OK;
}

template <typename T>
dd_status alloc_inner(dd_handle* h) {
  cplx<T>* q;
  const size_t nf = (size_t)h->nfine * h->nrhs;
  DD_TRY(h->alloc(&q, nf)); h->F = q;
  DD_TRY(h->alloc(&q, nf)); h->W = q;
  DD_TRY(h->alloc(&q, nf)); h->X = q;
  DD_TRY(h->alloc(&q, nf)); h->U = q;
  DD_TRY(h->alloc(&q, nf * (size_t)(h->maxit + 1))); h->V = q;
  return DD_OK;
}

template <typename T>
ddh::InnerArgs<T> inner_args(dd_handle* h) {
  ddh::InnerArgs<T> a{};
  a.subs = h->subs;
  a.order = h->order;
  a.cs = h->cs;
  a.local_bc = h->p.local_bc;
  a.fac = h->fac;
  a.Ec = h->Ec;
  a.F = (cplx<T>*)h->F;
  a.W = (cplx<T>*)h->W;
  a.X = (cplx<T>*)h->X;
  a.V = (cplx<T>*)h->V;
  a.R = h->R;
  a.Sc = h->Sc;
  a.iters = h->iters;
  a.flags = h->flags;
  a.counters = h->counters;
  a.nfine = h->nfine;
  a.ndof = h->ndof;
  a.rstride = h->ndof;
  a.zstride = h->ndof;
  a.nrhs = h->nrhs;
  a.maxit = h->maxit;
  a.max_nj = h->max_nj;
  a.max_nc = h->max_nc;
  a.tol = h->p.inner_tol;
  a.nt = h->inner_nt;
  a.order = h->lpt ? h->order : nullptr;
  return a;
}

// Guess tiles of the attached network for the subdomain right-hand sides R_j r (no-op
// without a network).
dd_status run_guess(dd_handle* h, const cplx<double>* r, long long rstride, const int* done, hipStream_t st,
                    const int* jdev = nullptr, long long rslot = 0) {
  if (!h->net || h->direct) return DD_OK;
  ddh::TileArgs ta{};
  ta.subs = h->subs;
  ta.cs = h->cs;
  ta.r = r;
  ta.rstride = rstride;
  ta.jdev = jdev;
  ta.rslot = rslot;
  ta.done = done;
  return ddh::net_infer_from(h->net, ta, h->nsub, h->nrhs, st);
}

// Batched subdomain solves: z = M^{-1} r over all right-hand sides (those with done set
// are skipped), starting from the network's guess tiles when a network is attached.
ddh::DirectArgs direct_args(dd_handle* h) {
  ddh::DirectArgs a{};
  a.subs = h->subs;
  a.order = h->lpt ? h->order : nullptr;
  a.cs = h->cs;
  a.local_bc = h->p.local_bc;
  a.ffac = h->ffac;
  a.foff = h->foff;
  a.iters = h->iters;
  a.flags = h->flags;
  a.counters = h->counters;
  a.nfine = h->nfine;
  a.ndof = h->ndof;
  a.rstride = h->ndof;
  a.zstride = h->ndof;
  a.nrhs = h->nrhs;
  a.max_nj = h->max_nj;
  return a;
}

dd_status run_inner(dd_handle* h, const cplx<double>* r, long long rstride, cplx<double>* z, long long zstride,
                    const int* done, hipStream_t st, const int* jdev = nullptr, long long rslot = 0,
                    long long zslot = 0, const cplx<double>* zadd = nullptr) {
  if (h->direct) {
    auto a = direct_args(h);
    a.r = r; a.z = z; a.done = done; a.rstride = rstride; a.zstride = zstride;
    a.jdev = jdev; a.rslot = rslot; a.zslot = zslot; a.zadd = zadd;
    DD_HIP(ddh::launch_direct_solve(a, st));
    return DD_OK;
  }
  if (h->multi) {
    ddh::MultiArgs a = h->mk;
    a.r = r; a.z = z; a.zadd = zadd; a.done = done;
    a.jdev = jdev; a.rslot = rslot; a.zslot = zslot;
    a.U = nullptr;
    (void)rstride; (void)zstride;   // one right-hand side
    DD_HIP(ddh::run_multi_inner(a, h->active_h, st));
    return DD_OK;
  }
  const float* gt = h->net ? h->net->y : nullptr;   // (exact solves take no guess)
  const int gT = h->net ? h->net->T : 0;
  if (h->prec == 32) {
    auto a = inner_args<float>(h);
    a.r = r; a.z = z; a.done = done; a.rstride = rstride; a.zstride = zstride;
    a.jdev = jdev; a.rslot = rslot; a.zslot = zslot; a.gtile = gt; a.gT = gT; a.zadd = zadd;
    DD_HIP(ddh::launch_inner_solve<float>(a, st));
  } else {
    auto a = inner_args<double>(h);
    a.r = r; a.z = z; a.done = done; a.rstride = rstride; a.zstride = zstride;
    a.jdev = jdev; a.rslot = rslot; a.zslot = zslot; a.gtile = gt; a.gT = gT; a.zadd = zadd;
    DD_HIP(ddh::launch_inner_solve<double>(a, st));
  }
  return DD_OK;
}

// Two-level coarse correction of the preconditioner input (no-op for the one-level
// method): q = Z_0 E_0^{-1} Z_0^T r and w = r - A q into the handle's coarse workspace.
dd_status run_coarse(dd_handle* h, const cplx<double>* r, long long rstride, const int* done, hipStream_t st,
                     const int* jdev = nullptr, long long rslot = 0) {
  if (!h->gc) return DD_OK;
  DD_HIP(h->gc->restrict_rhs(r, rstride, jdev, rslot, done, h->nrhs, st));
  DD_HIP(h->gc->solve(h->nrhs, st));
  DD_HIP(h->gc->correct(r, rstride, jdev, rslot, done, h->nrhs, st));
  return DD_OK;
}

// z = M^{-1} r: one-level (eq. 3), or two-level M_1^{-1} (r - A q) + q.
dd_status run_apply(dd_handle* h, const cplx<double>* r, long long rstride, cplx<double>* z, long long zstride,
                    const int* done, hipStream_t st) {
  DD_TRY(run_coarse(h, r, rstride, done, st));
  const cplx<double>* rin = h->gc ? h->gc->w : r;
  const long long rs = h->gc ? h->ndof : rstride;
  DD_TRY(run_guess(h, rin, rs, done, st));
  return run_inner(h, rin, rs, z, zstride, done, st, nullptr, 0, 0, h->gc ? h->gc->q : nullptr);
}

dd_status check_handle(const dd_handle* h) {
  if (!h) return fail(DD_EINVAL, "null handle");
  return DD_OK;
}

}  // namespace

extern "C" {

dd_status dd_setup(const dd_params* p, void* stream, dd_handle** out) {
  if (!p || !out) return fail(DD_EINVAL, "null argument");
  *out = nullptr;
  dd_handle* h = new dd_handle();
  dd_status s = validate_and_plan(p, h);
  if (s == DD_OK) s = h->prec == 32 ? check_lds<float>(h) : check_lds<double>(h);
  if (s != DD_OK) {
    delete h;
    return s;
  }
  hipStream_t st = (hipStream_t)stream;
  auto body = [&]() -> dd_status {
    DD_TRY(h->alloc(&h->subs, h->nsub));
    DD_HIP(hipMemcpy(h->subs, h->subs_h.data(), h->nsub * sizeof(SubDesc), hipMemcpyHostToDevice));
    // launch order: largest tiles first (longest-processing-time first), all right-hand sides
    std::vector<int> ord((size_t)h->nsub * h->nrhs);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
      const SubDesc& da = h->subs_h[a % h->nsub];
      const SubDesc& db = h->subs_h[b % h->nsub];
      return (long long)da.nx * da.ny > (long long)db.nx * db.ny;
    });
    DD_TRY(h->alloc(&h->order, ord.size()));
    DD_HIP(hipMemcpy(h->order, ord.data(), ord.size() * sizeof(int), hipMemcpyHostToDevice));
    DD_TRY(h->alloc(&h->Ec, (size_t)h->ncoarse * ddh::coarse_coefs(h->p.deflation)));
    DD_TRY(h->alloc(&h->fac, (size_t)h->nfac));
    DD_TRY(h->alloc(&h->pivmin, 2 * (size_t)h->nsub));
    DD_HIP(ddh::launch_assemble_coarse(h->subs, h->nsub, h->cs, h->p.local_bc, h->Ec, st));
    if (h->p.deflation == DD_DEFLATION_LINEAR)
      DD_HIP(ddh::launch_factor_coarse_twisted(h->subs, h->nsub, h->Ec, h->fac, h->pivmin, st));
    else
      DD_HIP(ddh::launch_factor_coarse_paired(h->subs, h->nsub, h->Ec, h->fac, h->pivmin, st));
    h->pivmin_h.resize(2 * (size_t)h->nsub);
    DD_HIP(hipMemcpyAsync(h->pivmin_h.data(), h->pivmin, 2 * h->nsub * sizeof(double), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < h->nsub; ++j)
      DD_TRY(check_pivots("coarse matrix E_" + std::to_string(j), h->pivmin_h[2 * j], h->pivmin_h[2 * j + 1]));
    if (h->direct) {
      // twisted block factorisation of every local matrix: its 9-coefficient form, factored by the same
      // kernel as E through per-subdomain views (block size nx, ny block rows)
      DD_TRY(h->alloc(&h->ffac, (size_t)h->nffac));
      DD_TRY(h->alloc(&h->foff, h->nsub));
      DD_HIP(hipMemcpy(h->foff, h->foff_h.data(), h->nsub * sizeof(long long), hipMemcpyHostToDevice));
      std::vector<SubDesc> views(h->subs_h);
      for (int j = 0; j < h->nsub; ++j) {
        views[j].mx = views[j].nx;
        views[j].my = views[j].ny;
        views[j].coff = views[j].off;
        views[j].goff = h->foff_h[j];
      }
      cplx<double>* Bc = nullptr;
      SubDesc* vd = nullptr;
      DD_HIP(hipMalloc((void**)&Bc, (size_t)h->nfine * 9 * sizeof(cplx<double>)));
      hipError_t e = hipMalloc((void**)&vd, h->nsub * sizeof(SubDesc));
      if (e == hipSuccess) e = hipMemcpy(vd, views.data(), h->nsub * sizeof(SubDesc), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = ddh::launch_fine_coef(h->subs, h->nsub, h->cs, h->p.local_bc, Bc, st);
      if (e == hipSuccess) e = ddh::launch_factor_coarse_twisted(vd, h->nsub, Bc, h->ffac, h->pivmin, st);
      if (e == hipSuccess) e = hipMemcpyAsync(h->pivmin_h.data(), h->pivmin, 2 * h->nsub * sizeof(double),
                                              hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      (void)hipFree(Bc);
      if (vd) (void)hipFree(vd);
      if (e != hipSuccess) return fail(DD_EHIP, std::string("direct factorisation: ") + hipGetErrorString(e));
      for (int j = 0; j < h->nsub; ++j)
        DD_TRY(check_pivots("local matrix B_" + std::to_string(j), h->pivmin_h[2 * j], h->pivmin_h[2 * j + 1]));
      DD_HIP(ddh::configure_direct(h->max_nj));
    }
    if (h->p.coarse_intervals > 0) {
      h->gc = new ddh::GlobalCoarse();
      const hipError_t e = h->gc->setup(h->n, h->p.coarse_intervals, h->p.k, h->nrhs, st);
      if (e != hipSuccess) return fail(DD_EHIP, std::string("global coarse set-up: ") + hipGetErrorString(e));
      DD_TRY(check_pivots("global coarse matrix E_0", h->gc->min_pivot, h->gc->max_entry));
    }
    if (h->prec == 32) DD_TRY(alloc_inner<float>(h));
    else DD_TRY(alloc_inner<double>(h));
    DD_TRY(h->alloc(&h->R, (size_t)h->nsub * h->nrhs * 2 * h->maxit * h->maxit));
    DD_TRY(h->alloc(&h->Sc, (size_t)h->nsub * h->nrhs * (h->maxit + 2) * h->max_nc));
    DD_TRY(h->alloc(&h->iters, (size_t)h->nsub * h->nrhs));
    DD_TRY(h->alloc(&h->flags, (size_t)h->nsub * h->nrhs));
    DD_TRY(h->alloc(&h->counters, 5));
    for (int e = 0; e < 8; ++e) DD_HIP(hipEventCreate(&h->ev[e]));
    h->ev_ok = true;
    // outer FGMRES workspaces
    const int m = h->restart;
    DD_TRY(h->alloc(&h->Vo, (size_t)h->nrhs * (m + 1) * h->ndof));
    DD_TRY(h->alloc(&h->Zo, (size_t)h->nrhs * m * h->ndof));
    h->pstride = 2 * m + 4;
    DD_TRY(h->alloc(&h->part, (size_t)h->nrhs * h->pstride *
                                  std::max<size_t>(ddh::outer_chunks(h->ndof),
                                                   ddh::dots2_chunks(h->ndof) + ddh::dots2_segments(h->ndof))));
    DD_TRY(h->alloc(&h->coef, (size_t)h->nrhs * h->pstride));
    DD_TRY(h->alloc(&h->ca, (size_t)h->nrhs * m));
    DD_TRY(h->alloc(&h->cb, (size_t)h->nrhs * m));
    DD_TRY(h->alloc(&h->scal, (size_t)h->nrhs * 4));
    ddh::OuterState& o = h->os;
    DD_TRY(h->alloc(&o.H, (size_t)h->nrhs * (m + 1)));
    DD_TRY(h->alloc(&o.cs, (size_t)h->nrhs * m));
    DD_TRY(h->alloc(&o.sn, (size_t)h->nrhs * m));
    DD_TRY(h->alloc(&o.g, (size_t)h->nrhs * (m + 1)));
    DD_TRY(h->alloc(&o.R, (size_t)h->nrhs * m * m));
    DD_TRY(h->alloc(&o.y, (size_t)h->nrhs * m));
    DD_TRY(h->alloc(&o.res, h->nrhs));
    DD_TRY(h->alloc(&o.hnext, h->nrhs));
    DD_TRY(h->alloc(&o.atol, h->nrhs));
    DD_TRY(h->alloc(&o.steps, h->nrhs));
    DD_TRY(h->alloc(&o.done, h->nrhs));
    DD_TRY(h->alloc(&o.applies, h->nrhs));
    DD_TRY(h->alloc(&o.sweep_bytes, 2));
    DD_TRY(h->alloc(&h->jdev, 1));
    const int slots = std::max(1, h->p.graph_steps);
    h->sev.resize((size_t)slots * kEvPerStep);
    for (auto& e : h->sev) DD_HIP(hipEventCreate(&e));
    if (h->prec == 32) DD_HIP(ddh::configure_inner<float>(h->max_nj, h->max_nc, h->maxit));
    else DD_HIP(ddh::configure_inner<double>(h->max_nj, h->max_nc, h->maxit));
    DD_HIP(ddh::configure_outer());
    o.nrm2 = h->coef;
    o.nrm_stride = h->pstride;
    o.rtol = h->p.outer_tol;
    o.restart = m;
    DD_HIP(hipHostMalloc((void**)&h->done_h, h->nrhs * sizeof(int), hipHostMallocDefault));
    DD_HIP(hipHostMalloc((void**)&h->res_h, h->nrhs * sizeof(double), hipHostMallocDefault));
    if (h->multi) {
      ddh::MultiArgs& a = h->mk;
      const size_t nf = (size_t)h->nfine, nc = (size_t)h->ncoarse, ns = (size_t)h->nsub, m = (size_t)h->maxit;
      a.subs = h->subs;
      a.cs = h->cs;
      a.local_bc = h->p.local_bc;
      a.fac = h->fac;
      a.Ec = h->Ec;
      a.F = (cplx<double>*)h->F;
      a.W = (cplx<double>*)h->W;
      a.X = (cplx<double>*)h->X;
      a.V = (cplx<double>*)h->V;
      a.R = h->R;
      a.iters = h->iters;
      a.flags = h->flags;
      a.counters = h->counters;
      DD_TRY(h->alloc(&a.T, nf));
      DD_TRY(h->alloc(&a.Bv, nf));
      DD_TRY(h->alloc(&a.Zc, nf));
      DD_TRY(h->alloc(&a.t, nc));
      DD_TRY(h->alloc(&a.Cv, nc));
      DD_TRY(h->alloc(&a.Yk, (m + 2) * nc));
      DD_TRY(h->alloc(&a.H, ns * (m + 1)));
      DD_TRY(h->alloc(&a.g, ns * (m + 1)));
      DD_TRY(h->alloc(&a.csn, ns * m));
      DD_TRY(h->alloc(&a.snn, ns * m));
      DD_TRY(h->alloc(&a.fnorm, ns));
      DD_TRY(h->alloc(&a.ref, ns));
      DD_TRY(h->alloc(&a.wn, ns));
      DD_TRY(h->alloc(&a.active, ns));
      DD_TRY(h->alloc(&a.notconv, ns));
      DD_TRY(h->alloc(&a.nactive, 1));
      a.nfine = h->nfine;
      a.ncoarse = h->ncoarse;
      a.nsub = h->nsub;
      a.maxit = h->maxit;
      a.max_nj = h->max_nj;
      a.max_nc = h->max_nc;
      a.tol = h->p.inner_tol;
      DD_HIP(hipHostMalloc((void**)&h->active_h, sizeof(int), hipHostMallocDefault));
    }
    return DD_OK;
  };
  s = body();
  if (s != DD_OK) {
    h->release();
    delete h;
    return s;
  }
  *out = h;
  return DD_OK;
}

dd_status dd_destroy(dd_handle* h) {
  if (!h) return DD_OK;
  h->release();
  delete h;
  return DD_OK;
}

dd_status dd_set_graph(dd_handle* h, int use_graph) {
  DD_TRY(check_handle(h));
  if (use_graph && (h->p.graph_steps < 1 || h->p.graph_steps > kMaxGraphSteps))
    return fail(DD_EINVAL, "graph_steps must be in [1, 64]");
  if (use_graph && h->multi) return fail(DD_EINVAL, "the multi-launch form cannot be graph-captured");
  h->p.use_graph = use_graph ? 1 : 0;
  return DD_OK;
}

int64_t dd_num_dofs(const dd_handle* h) { return h ? h->ndof : 0; }
int dd_num_subdomains(const dd_handle* h) { return h ? h->nsub : 0; }
int dd_num_intervals(const dd_handle* h) { return h ? h->n : 0; }
int64_t dd_packed_fine_size(const dd_handle* h) { return h ? h->nfine : 0; }
int64_t dd_packed_coarse_size(const dd_handle* h) { return h ? h->ncoarse : 0; }

dd_status dd_layout(const dd_handle* h, int32_t* out) {
  DD_TRY(check_handle(h));
  if (!out) return fail(DD_EINVAL, "null output");
  for (int j = 0; j < h->nsub; ++j) {
    const SubDesc& d = h->subs_h[j];
    int32_t* o = out + 12 * j;
    o[0] = d.i0; o[1] = d.j0; o[2] = d.nx; o[3] = d.ny;
    o[4] = d.ax; o[5] = d.bx; o[6] = d.ay; o[7] = d.by;
    o[8] = d.mx; o[9] = d.my; o[10] = (int32_t)d.off; o[11] = (int32_t)d.coff;
  }
  return DD_OK;
}

dd_status dd_coarse_matrix(const dd_handle* h, int j, double* out, double* min_pivot) {
  DD_TRY(check_handle(h));
  if (j < 0 || j >= h->nsub || !out) return fail(DD_EINVAL, "bad subdomain index or null output");
  const SubDesc& d = h->subs_h[j];
  const int K = ddh::coarse_coefs(h->p.deflation);
  DD_HIP(hipMemcpy(out, h->Ec + d.coff * K, (size_t)d.mx * d.my * K * sizeof(cplx<double>), hipMemcpyDeviceToHost));
  if (min_pivot) *min_pivot = h->pivmin_h[2 * (size_t)j];
  return DD_OK;
}

dd_status dd_apply_preconditioner(dd_handle* h, const void* r, void* z, void* stream) {
  DD_TRY(check_handle(h));
  if (!r || !z || r == z) return fail(DD_EINVAL, "r and z must be distinct non-null device pointers");
  return run_apply(h, (const cplx<double>*)r, h->ndof, (cplx<double>*)z, h->ndof, nullptr, (hipStream_t)stream);
}

// One outer FGMRES step j (j read from h->jdev by every kernel): z_j = M^{-1} v~_j,
// w = A z_j, delayed-CGS2 dot sweep + bookkeeping + update sweep, j += 1.  Right-hand
// sides whose done flag is set skip all of it.  `slot` selects the phase events.
static dd_status enqueue_outer_step(dd_handle* h, int slot, hipStream_t st, bool timed) {
  const int m = h->restart, nr = h->nrhs;
  const long long nd = h->ndof;
  const long long vstr = (long long)(m + 1) * nd, zstr = (long long)m * nd;
  ddh::OuterState& o = h->os;
  const ddh::StepRef sr = ddh::device_step(h->jdev);
  hipEvent_t* ev = h->sev.data() + (size_t)slot * kEvPerStep;
  auto mark = [&](int e) -> dd_status {
    if (timed) DD_HIP(hipEventRecord(ev[e], st));
    return DD_OK;
  };
  DD_TRY(mark(0));
  DD_TRY(run_coarse(h, h->Vo, vstr, o.done, st, h->jdev, nd));
  DD_TRY(mark(1));
  if (h->gc) DD_TRY(run_guess(h, h->gc->w, nd, o.done, st));
  else DD_TRY(run_guess(h, h->Vo, vstr, o.done, st, h->jdev, nd));
  DD_TRY(mark(2));
  if (h->gc) DD_TRY(run_inner(h, h->gc->w, nd, h->Zo, zstr, o.done, st, h->jdev, 0, nd, h->gc->q));
  else DD_TRY(run_inner(h, h->Vo, vstr, h->Zo, zstr, o.done, st, h->jdev, nd, nd));
  DD_TRY(mark(3));
  DD_HIP(ddh::launch_global_apply_masked(h->cs, h->Zo, zstr, h->Vo + nd, vstr, nr, o.done, st, sr, nd, nd));
  DD_TRY(mark(4));
  DD_HIP(ddh::launch_dots2(h->Vo, vstr, nullptr, 0, nullptr, 0, nd, sr, 1, m, h->part, h->pstride, nr, o.done, st,
                           h->dots_blocks));
  DD_TRY(mark(5));
  DD_HIP(ddh::launch_reduce_chunks(h->part, nd, h->pstride, sr, 2, 3, m, h->coef, h->pstride, nr, o.done, st));
  DD_HIP(ddh::launch_dcgs2_step(o, sr, m, nd, h->coef, h->pstride, 1, h->ca, h->cb, m, h->scal, nr, st));
  DD_TRY(mark(6));
  DD_HIP(ddh::launch_dcgs2_update(h->Vo, vstr, nd, sr, h->ca, h->cb, m, h->scal, nr, o.done, st));
  DD_TRY(mark(7));
  DD_HIP(ddh::launch_advance_step(h->jdev, st));
  return DD_OK;
}

// Capture graph_steps consecutive outer steps once per handle (on a private stream:
// the caller's stream may be the legacy default stream, which cannot be captured).
static dd_status ensure_graph(dd_handle* h) {
  if (h->graph_exec) return DD_OK;
  if (!h->cap_stream) DD_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  DD_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  dd_status s = DD_OK;
  for (int q = 0; q < h->p.graph_steps && s == DD_OK; ++q) s = enqueue_outer_step(h, q, h->cap_stream, false);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (s != DD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(DD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  h->graph = g;
  DD_HIP(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
  return DD_OK;
}

dd_status dd_solve(dd_handle* h, const void* fv, void* uv, void* stream, dd_stats* stats) {
  DD_TRY(check_handle(h));
  if (!fv || !uv || fv == uv) return fail(DD_EINVAL, "f and u must be distinct non-null device pointers");
  hipStream_t st = (hipStream_t)stream;
  const cplx<double>* f = (const cplx<double>*)fv;
  cplx<double>* u = (cplx<double>*)uv;
  const int m = h->restart, nr = h->nrhs;
  const long long nd = h->ndof;
  const long long vstr = (long long)(m + 1) * nd, zstr = (long long)m * nd;
  ddh::OuterState& o = h->os;
  const int S = h->p.use_graph ? h->p.graph_steps : 1;
  if (h->p.use_graph) DD_TRY(ensure_graph(h));
  DD_HIP(hipMemsetAsync(h->counters, 0, 5 * sizeof(unsigned long long), st));
  DD_HIP(hipMemsetAsync(o.applies, 0, nr * sizeof(int), st));
  DD_HIP(hipMemsetAsync(o.sweep_bytes, 0, 2 * sizeof(unsigned long long), st));
  DD_HIP(hipMemsetAsync(u, 0, (size_t)nr * nd * sizeof(cplx<double>), st));
  // coarse correction, guess, inner, global stencil, dot sweep, bookkeeping, update sweep
  double ms[7] = {0, 0, 0, 0, 0, 0, 0};
  double ms_steps = 0.0;            // all outer steps (graph replays and eager steps)
  int launches = 0, replays = 0, timed_steps = 0;
  float el = 0.f;
  int steps_run = 0, columns = 0;
  bool all_done = false;
  std::vector<int> steps_h(nr);
  o.first_cycle = 1;
  // r0 = f  (u = 0)
  DD_HIP(hipMemcpy2DAsync(h->Vo, vstr * sizeof(cplx<double>), f, nd * sizeof(cplx<double>),
                          nd * sizeof(cplx<double>), nr, hipMemcpyDeviceToDevice, st));
  auto sync_done = [&]() -> dd_status {
    DD_HIP(hipMemcpyAsync(h->done_h, o.done, nr * sizeof(int), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    all_done = true;
    for (int q = 0; q < nr; ++q) all_done = all_done && h->done_h[q];
    return DD_OK;
  };
  while (true) {
    // beta = ||r||, g = (beta, 0, ..), v~_0 = r / beta, j = 0
    DD_HIP(ddh::launch_dots(h->Vo, vstr, h->Vo, vstr, nd, 0, 1, h->part, h->pstride, nr, nullptr, st));
    DD_HIP(ddh::launch_reduce_parts(h->part, ddh::outer_chunks(nd), h->pstride, ddh::host_step(0), 0, 1, 0, h->coef,
                                    h->pstride, nullptr, 0, 2, nr, nullptr, st));
    DD_HIP(ddh::launch_cycle_init(o, nr, st));
    DD_HIP(ddh::launch_scale(h->Vo, vstr, h->Vo, vstr, nd, o.hnext, kOuterBlocks, nr, o.done, st));
    DD_HIP(hipMemsetAsync(h->jdev, 0, sizeof(int), st));
    o.first_cycle = 0;
    DD_TRY(sync_done());
    if (all_done) break;
    int j = 0;
    while (j < m && steps_run < h->p.outer_maxit) {
      const int batch = std::min(S, std::min(m - j, h->p.outer_maxit - steps_run));
      const bool replay = h->p.use_graph && batch == S;
      DD_HIP(hipEventRecord(h->ev[0], st));
      if (replay) {
        DD_HIP(hipGraphLaunch(h->graph_exec, st));
        ++replays;
      } else {
        for (int q = 0; q < batch; ++q) DD_TRY(enqueue_outer_step(h, q, st, true));
      }
      DD_HIP(hipEventRecord(h->ev[1], st));
      j += batch;
      steps_run += batch;
      launches += batch;
      DD_TRY(sync_done());
      DD_HIP(hipEventElapsedTime(&el, h->ev[0], h->ev[1]));
      ms_steps += el;
      if (!replay) {
        timed_steps += batch;
        for (int q = 0; q < batch; ++q) {
          hipEvent_t* ev = h->sev.data() + (size_t)q * kEvPerStep;
          for (int e = 0; e < 7; ++e) {
            DD_HIP(hipEventElapsedTime(&el, ev[e], ev[e + 1]));
            ms[e] += el;
          }
        }
      }
      if (all_done) break;
    }
    if (!all_done && j == m) {
      // end of a cycle: finalise column m-1 from v~_m alone
      DD_HIP(ddh::launch_dots2(h->Vo, vstr, h->Vo + (long long)m * nd, vstr, nullptr, 0, nd, ddh::host_step(m), 0, m,
                               h->part, h->pstride, nr, o.done, st, h->dots_blocks));
      DD_HIP(ddh::launch_reduce_chunks(h->part, nd, h->pstride, ddh::host_step(m), 2, 3, m, h->coef, h->pstride, nr,
                                       o.done, st));
      DD_HIP(ddh::launch_dcgs2_step(o, ddh::host_step(m), m, nd, h->coef, h->pstride, 0, h->ca, h->cb, m, h->scal,
                                    nr, st));
      DD_TRY(sync_done());
    }
    // u += Z y over the columns each right-hand side finalised in this cycle
    DD_HIP(ddh::launch_backsolve(o, nr, st));
    DD_HIP(hipMemcpyAsync(steps_h.data(), o.steps, nr * sizeof(int), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    const int kmax = *std::max_element(steps_h.begin(), steps_h.end());
    columns += kmax;
    DD_HIP(ddh::launch_update(h->Zo, zstr, u, nd, nd, kmax, o.y, m, 1.0, nr, nullptr, st));
    if (all_done || steps_run >= h->p.outer_maxit) break;
    // restart: r = f - A u
    DD_HIP(ddh::launch_global_apply_masked(h->cs, u, nd, h->Vo, vstr, nr, nullptr, st));
    DD_HIP(ddh::launch_residual(f, nd, h->Vo, vstr, nd, kOuterBlocks, nr, st));
  }
  if (stats) {
    unsigned long long c[5], sb[2];
    std::vector<int> app(nr);
    DD_HIP(hipMemcpyAsync(c, h->counters, sizeof(c), hipMemcpyDeviceToHost, st));
    DD_HIP(hipMemcpyAsync(sb, o.sweep_bytes, sizeof(sb), hipMemcpyDeviceToHost, st));
    DD_HIP(hipMemcpyAsync(app.data(), o.applies, nr * sizeof(int), hipMemcpyDeviceToHost, st));
    DD_HIP(hipMemcpyAsync(h->res_h, o.res, nr * sizeof(double), hipMemcpyDeviceToHost, st));
    std::vector<double> at(nr);
    DD_HIP(hipMemcpyAsync(at.data(), o.atol, nr * sizeof(double), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    stats->outer_iters = columns;
    stats->precond_applies = *std::max_element(app.begin(), app.end());
    stats->converged = all_done ? 1 : 0;
    stats->inner_iters_total = (long long)c[0];
    stats->subdomain_solves = (long long)c[1];
    stats->inner_iters_max = (int)c[2];
    stats->guesses_accepted = (long long)c[3];
    stats->inner_bytes = (double)c[4];
    stats->ms_coarse = ms[0];
    stats->coarse_bytes = h->gc ? (double)h->gc->solve_bytes() : 0.0;
    stats->ms_guess = ms[1];
    stats->ms_inner = ms[2];
    stats->ms_spmv = ms[3];
    stats->ms_orth = ms[4] + ms[5] + ms[6];
    stats->ms_other = ms[5];
    stats->ms_dots = ms[4];
    stats->ms_update = ms[6];
    stats->dots_bytes = (double)sb[0];
    stats->update_bytes = (double)sb[1];
    stats->inner_launches = launches;
    stats->graph_replays = replays;
    stats->timed_steps = timed_steps;
    stats->ms_steps = ms_steps;
    double worst = 0.0;
    for (int q = 0; q < nr; ++q) {
      const double rel = at[q] > 0 ? h->res_h[q] / (at[q] / h->p.outer_tol) : 0.0;
      worst = std::max(worst, rel);
    }
    stats->final_res_estimate = worst;
  }
  return all_done ? DD_OK : fail(DD_ENOTCONV, "outer FGMRES reached outer_maxit");
}

// ---- autotuner ---------------------------------------------------------------------

static std::string tune_signature(const dd_handle* h) {
  hipDeviceProp_t prop{};
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  unsigned long long hc = 1469598103934665603ull;   // FNV-1a over the cut points
  auto mix = [&](long long v) { hc = (hc ^ (unsigned long long)v) * 1099511628211ull; };
  for (int c : h->cuts_x) mix(c);
  for (int c : h->cuts_y) mix(c + 1000003);
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "%s N=%d px=%d py=%d cuts=%016llx ov=%d bc=%d prec=%d maxit=%d nrhs=%d m=%d ls=%d M0=%d",
                prop.gcnArchName, h->n, h->p.px, h->p.py, hc, h->p.overlap, h->p.local_bc, h->prec, h->maxit,
                h->nrhs, h->restart, h->p.local_solver, h->p.coarse_intervals);
  return buf;
}

static void invalidate_graph(dd_handle* h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
}

extern "C" dd_status dd_autotune(dd_handle* h, const char* cache_path, void* stream, char* report, int report_len) {
  DD_TRY(check_handle(h));
  if (h->multi) return fail(DD_EINVAL, "the multi-launch form has no launch configuration to tune");
  hipStream_t st = (hipStream_t)stream;
  const std::string sig = tune_signature(h);
  std::string rep;
  auto finish = [&](const std::string& how) -> dd_status {
    char b[256];
    std::snprintf(b, sizeof(b), "%s: inner_threads=%d lpt=%d dots_blocks=%d", how.c_str(), h->inner_nt,
                  h->lpt ? 1 : 0, h->dots_blocks);
    rep = std::string(b) + rep;
    if (report && report_len > 0) {
      std::snprintf(report, (size_t)report_len, "%s", rep.c_str());
    }
    invalidate_graph(h);
    return DD_OK;
  };
  if (cache_path) {
    FILE* fp = std::fopen(cache_path, "r");
    if (fp) {
      char line[1024];
      while (std::fgets(line, sizeof(line), fp)) {
        std::string l(line);
        const size_t bar = l.find(" | ");
        if (bar == std::string::npos || l.substr(0, bar) != sig) continue;
        int nt = 0, lp = 1, db = 0;
        if (std::sscanf(l.c_str() + bar + 3, "inner_threads=%d lpt=%d dots_blocks=%d", &nt, &lp, &db) == 3 &&
            (nt == 256 || nt == 512)) {
          h->inner_nt = nt;
          h->lpt = lp != 0;
          h->dots_blocks = db;
          std::fclose(fp);
          return finish("cache");
        }
      }
      std::fclose(fp);
    }
  }
  const int m = h->restart;
  const long long nd = h->ndof;
  const long long vstr = (long long)(m + 1) * nd, zstr = (long long)m * nd;
  // the events are destroyed on every return path
  struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  DD_HIP(hipEventCreate(&ev.a));
  DD_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  auto time_ms = [&](auto&& fn, int reps) -> double {
    std::vector<float> t;
    for (int r = 0; r < reps + 1; ++r) {
      (void)hipEventRecord(e0, st);
      fn();
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      float x = 0.f;
      (void)hipEventElapsedTime(&x, e0, e1);
      if (r > 0) t.push_back(x);   // first run warms up
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
  };
  // representative data: pseudo-random residual in slot 0 (and basis vectors for the sweep);
  // the basis has slots 0..m, and a dot sweep at step jj reads slots 0..jj+1, so jj <= m - 1
  const int jt = std::max(0, std::min(m - 1, 1024));
  for (int q = 0; q < h->nrhs; ++q)
    DD_HIP(ddh::launch_fill_hash(h->Vo + q * vstr, (long long)(jt + 2) * nd, 17081ull + q, st));
  double best = 1e300;
  int best_nt = h->inner_nt;
  bool best_lpt = h->lpt;
  char line[160];
  for (int nt : {512, 256}) {
    for (bool lp : {true, false}) {
      h->inner_nt = nt;
      h->lpt = lp;
      dd_status s = DD_OK;
      const double ms = time_ms([&]() { s = run_apply(h, h->Vo, vstr, h->Zo, zstr, nullptr, st); }, 3);
      if (s != DD_OK) return s;
      std::snprintf(line, sizeof(line), "\n  inner_threads=%d lpt=%d: %.3f ms per preconditioner application", nt,
                    lp ? 1 : 0, ms);
      rep += line;
      if (ms < best) { best = ms; best_nt = nt; best_lpt = lp; }
    }
  }
  h->inner_nt = best_nt;
  h->lpt = best_lpt;
  double bestd = 1e300;
  int best_db = 0;
  // the sweep's cost grows with the basis: time it at a short and a long basis (with a
  // restart length below 2 there is no sweep worth tuning and the default stays)
  const int jshort = std::max(1, jt / 4);
  for (int db : {1024, 2048, 4096, 8192, 16384}) {
    if (jt < 1) break;
    const double ms = time_ms([&]() {
      for (int jj : {jshort, jt})
        (void)ddh::launch_dots2(h->Vo, vstr, h->Vo + (long long)jj * nd, vstr, h->Vo + (long long)(jj + 1) * nd, vstr,
                                nd, ddh::host_step(jj), 1, jj, h->part, h->pstride, h->nrhs, nullptr, st, db);
    }, 3);
    std::snprintf(line, sizeof(line), "\n  dots_blocks=%d: %.3f ms for dot sweeps over %d and %d vectors", db, ms,
                  jshort, jt);
    rep += line;
    if (ms < bestd) { bestd = ms; best_db = db; }
  }
  if (jt >= 1) h->dots_blocks = best_db;
  DD_HIP(hipGetLastError());
  if (cache_path) {
    FILE* fp = std::fopen(cache_path, "a");
    if (fp) {
      std::fprintf(fp, "%s | inner_threads=%d lpt=%d dots_blocks=%d\n", sig.c_str(), h->inner_nt, h->lpt ? 1 : 0,
                   h->dots_blocks);
      std::fclose(fp);
    }
  }
  return finish("measured");
}

// ---- kernel-level entry points -----------------------------------------------------

dd_status dd_op_global_apply(dd_handle* h, const void* v, void* w, void* stream) {
  DD_TRY(check_handle(h));
  if (!v || !w) return fail(DD_EINVAL, "null vector");
  DD_HIP(ddh::launch_global_apply(h->cs, (const cplx<double>*)v, (cplx<double>*)w, 1, (hipStream_t)stream));
  return DD_OK;
}

dd_status dd_op_local_apply(dd_handle* h, int precision, const void* v, void* w, void* stream) {
  DD_TRY(check_handle(h));
  if (!v || !w) return fail(DD_EINVAL, "null vector");
  hipStream_t st = (hipStream_t)stream;
  if (precision == 32)
    DD_HIP(ddh::launch_local_apply<float>(h->subs, h->nsub, h->cs, h->p.local_bc, (const cplx<float>*)v,
                                          (cplx<float>*)w, h->max_nj, st));
  else if (precision == 64)
    DD_HIP(ddh::launch_local_apply<double>(h->subs, h->nsub, h->cs, h->p.local_bc, (const cplx<double>*)v,
                                           (cplx<double>*)w, h->max_nj, st));
  else
    return fail(DD_EINVAL, "precision must be 32 or 64");
  return DD_OK;
}

dd_status dd_op_deflated_apply(dd_handle* h, int precision, const void* v, void* w, void* stream) {
  DD_TRY(check_handle(h));
  if (!v || !w) return fail(DD_EINVAL, "null vector");
  hipStream_t st = (hipStream_t)stream;
  if (precision == 32)
    DD_HIP(ddh::launch_deflated_apply<float>(h->subs, h->nsub, h->cs, h->p.local_bc, h->fac, h->Ec,
                                             (const cplx<float>*)v, (cplx<float>*)w, h->max_nj, h->max_nc, st));
  else if (precision == 64)
    DD_HIP(ddh::launch_deflated_apply<double>(h->subs, h->nsub, h->cs, h->p.local_bc, h->fac, h->Ec,
                                              (const cplx<double>*)v, (cplx<double>*)w, h->max_nj, h->max_nc, st));
  else
    return fail(DD_EINVAL, "precision must be 32 or 64");
  return DD_OK;
}

dd_status dd_op_restrict(dd_handle* h, const void* v, void* t, void* stream) {
  DD_TRY(check_handle(h));
  if (!v || !t) return fail(DD_EINVAL, "null vector");
  DD_HIP(ddh::launch_restrict(h->subs, h->nsub, (const cplx<double>*)v, (cplx<double>*)t, (hipStream_t)stream));
  return DD_OK;
}

dd_status dd_op_prolong(dd_handle* h, const void* y, void* v, void* stream) {
  DD_TRY(check_handle(h));
  if (!v || !y) return fail(DD_EINVAL, "null vector");
  DD_HIP(ddh::launch_prolong(h->subs, h->nsub, (const cplx<double>*)y, (cplx<double>*)v, (hipStream_t)stream));
  return DD_OK;
}

dd_status dd_op_coarse_solve(dd_handle* h, const void* t, void* y, void* stream) {
  DD_TRY(check_handle(h));
  if (!t || !y || t == y) return fail(DD_EINVAL, "t and y must be distinct non-null vectors");
  DD_HIP(ddh::launch_coarse_solve(h->subs, h->nsub, h->fac, h->Ec, (const cplx<double>*)t, (cplx<double>*)y,
                                  h->max_nc, (hipStream_t)stream));
  return DD_OK;
}

dd_status dd_op_gather(dd_handle* h, int precision, const void* r, void* f, void* stream) {
  DD_TRY(check_handle(h));
  if (!r || !f) return fail(DD_EINVAL, "null vector");
  hipStream_t st = (hipStream_t)stream;
  if (precision == 32)
    DD_HIP(ddh::launch_gather<float>(h->subs, h->nsub, h->cs, (const cplx<double>*)r, (cplx<float>*)f, h->nfine,
                                     h->ndof, 1, st));
  else if (precision == 64)
    DD_HIP(ddh::launch_gather<double>(h->subs, h->nsub, h->cs, (const cplx<double>*)r, (cplx<double>*)f, h->nfine,
                                      h->ndof, 1, st));
  else
    return fail(DD_EINVAL, "precision must be 32 or 64");
  return DD_OK;
}

dd_status dd_op_scatter(dd_handle* h, int precision, const void* u, void* z, void* stream) {
  DD_TRY(check_handle(h));
  if (!u || !z) return fail(DD_EINVAL, "null vector");
  hipStream_t st = (hipStream_t)stream;
  if (precision == 32)
    DD_HIP(ddh::launch_scatter<float>(h->subs, h->nsub, h->cs, (const cplx<float>*)u, (cplx<double>*)z, h->nfine,
                                      h->ndof, 1, st));
  else if (precision == 64)
    DD_HIP(ddh::launch_scatter<double>(h->subs, h->nsub, h->cs, (const cplx<double>*)u, (cplx<double>*)z,
                                       h->nfine, h->ndof, 1, st));
  else
    return fail(DD_EINVAL, "precision must be 32 or 64");
  return DD_OK;
}

dd_status dd_op_inner_solve(dd_handle* h, const void* f, const void* guess, void* u, int32_t* iters, int32_t* flags,
                            void* stream) {
  DD_TRY(check_handle(h));
  if (!f || !u) return fail(DD_EINVAL, "null vector");
  if (h->multi && guess) return fail(DD_EINVAL, "the multi-launch form takes no initial guess");
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = (size_t)h->nfine * h->nrhs * (h->prec == 32 ? 8 : 16);
  DD_HIP(hipMemcpyAsync(h->F, f, bytes, hipMemcpyDeviceToDevice, st));
  if (h->direct) {
    auto a = direct_args(h);
    a.F = (const cplx<double>*)h->F;
    a.U = (cplx<double>*)u;
    DD_HIP(ddh::launch_direct_solve(a, st));
  } else if (h->multi) {
    ddh::MultiArgs a = h->mk;
    a.U = (cplx<double>*)u;
    DD_HIP(ddh::run_multi_inner(a, h->active_h, st));
  } else if (h->prec == 32) {
    auto a = inner_args<float>(h);
    a.guess = (const cplx<float>*)guess;
    a.U = (cplx<float>*)u;
    DD_HIP(ddh::launch_inner_solve<float>(a, st));
  } else {
    auto a = inner_args<double>(h);
    a.guess = (const cplx<double>*)guess;
    a.U = (cplx<double>*)u;
    DD_HIP(ddh::launch_inner_solve<double>(a, st));
  }
  const size_t cnt = (size_t)h->nsub * h->nrhs;
  if (iters) DD_HIP(hipMemcpyAsync(iters, h->iters, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
  if (flags) DD_HIP(hipMemcpyAsync(flags, h->flags, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

// Batched subdomain solves with every scratch buffer in the library's static device array
// (allocates nothing; see include/ddhelm.h).
extern "C++" template <typename T>
static dd_status inner_solve_static(dd_handle* h, const void* f, void* u, int32_t* iters, int32_t* flags,
                                    hipStream_t st) {
  void* base = nullptr;
  size_t cap = 0;
  DD_HIP(ddh::static_scratch(&base, &cap));
  const size_t ns = (size_t)h->nsub * h->nrhs, nf = (size_t)h->nfine * h->nrhs, mi = (size_t)h->maxit;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t off = 0;
  auto take = [&](size_t b) { const size_t o = off; off += up(b); return o; };
  const size_t o_cnt = take(5 * sizeof(unsigned long long));
  const size_t o_it = take(ns * sizeof(int));
  const size_t o_fl = take(ns * sizeof(int));
  const size_t o_v = take(nf * (mi + 1) * sizeof(cplx<T>));
  const size_t o_w = take(nf * sizeof(cplx<T>));
  const size_t o_x = take(nf * sizeof(cplx<T>));
  const size_t o_r = take(ns * 2 * mi * mi * sizeof(cplx<double>));
  const size_t o_sc = take(ns * (mi + 2) * (size_t)h->max_nc * sizeof(cplx<double>));
  if (off > cap)
    return fail(DD_EINVAL, "the subdomain solves of this handle need " + std::to_string(off) +
                               " bytes of scratch; the static scratch holds " + std::to_string(cap) +
                               " (lower inner_maxit or the problem size, or use dd_op_inner_solve)");
  unsigned char* b = (unsigned char*)base;
  auto a = inner_args<T>(h);
  a.F = (cplx<T>*)const_cast<void*>(f);   // read only: with no global residual the kernel reads F
  a.U = (cplx<T>*)u;
  a.guess = nullptr;
  a.gtile = nullptr;
  a.counters = (unsigned long long*)(b + o_cnt);
  a.iters = (int*)(b + o_it);
  a.flags = (int*)(b + o_fl);
  a.V = (cplx<T>*)(b + o_v);
  a.W = (cplx<T>*)(b + o_w);
  a.X = (cplx<T>*)(b + o_x);
  a.R = (cplx<double>*)(b + o_r);
  a.Sc = (cplx<double>*)(b + o_sc);
  DD_HIP(ddh::launch_zero_words(a.counters, 5, st));   // the array keeps the previous call's contents
  DD_HIP(ddh::launch_inner_solve<T>(a, st));
  if (iters) DD_HIP(hipMemcpyAsync(iters, a.iters, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  if (flags) DD_HIP(hipMemcpyAsync(flags, a.flags, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  if (iters || flags) DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

dd_status dd_op_inner_solve_static(dd_handle* h, const void* f, void* u, int32_t* iters, int32_t* flags,
                                   void* stream) {
  DD_TRY(check_handle(h));
  if (!f || !u || f == u) return fail(DD_EINVAL, "f and u must be distinct non-null device pointers");
  if (h->direct || h->multi)
    return fail(DD_EINVAL, "the static-scratch subdomain solves need the fused deflated-GMRES form "
                           "(local_solver DD_LOCAL_DEFLATED_GMRES, inner_launch DD_INNER_FUSED)");
  hipStream_t st = (hipStream_t)stream;
  return h->prec == 32 ? inner_solve_static<float>(h, f, u, iters, flags, st)
                       : inner_solve_static<double>(h, f, u, iters, flags, st);
}

// ---- learned initial guess ---------------------------------------------------------------

dd_status dd_set_guess(dd_handle* h, dd_net* net) {
  DD_TRY(check_handle(h));
  if (net && h->multi) return fail(DD_EINVAL, "the multi-launch form takes no guess network");
  if (net) {
    for (const SubDesc& d : h->subs_h)
      if (d.nx > net->T || d.ny > net->T)
        return fail(DD_EINVAL, "network tile " + std::to_string(net->T) + " smaller than a subdomain tile (" +
                                   std::to_string(d.nx) + " x " + std::to_string(d.ny) + ")");
    if ((long long)h->nsub * h->nrhs > net->B)
      return fail(DD_EINVAL, "network max_batch smaller than nsub * nrhs");
  }
  if (net != h->net) invalidate_graph(h);
  h->net = net;
  return DD_OK;
}

dd_status dd_tiles(dd_handle* h, const void* r, int tile, float* x, double* scale, void* stream) {
  DD_TRY(check_handle(h));
  if (!r || !x || !scale) return fail(DD_EINVAL, "null argument");
  for (const SubDesc& d : h->subs_h)
    if (d.nx > tile || d.ny > tile) return fail(DD_EINVAL, "tile smaller than a subdomain tile");
  ddh::TileArgs ta{};
  ta.subs = h->subs;
  ta.cs = h->cs;
  ta.r = (const cplx<double>*)r;
  ta.rstride = h->ndof;
  ta.T = tile;
  ta.xf = x;
  ta.scale = scale;
  DD_HIP(ddh::launch_tiles(ta, h->nsub, h->nrhs, (hipStream_t)stream));
  return DD_OK;
}

dd_status dd_packed_to_tiles(dd_handle* h, const void* u, const double* scale, int tile, float* t, void* stream) {
  DD_TRY(check_handle(h));
  if (!u || !scale || !t) return fail(DD_EINVAL, "null argument");
  for (const SubDesc& d : h->subs_h)
    if (d.nx > tile || d.ny > tile) return fail(DD_EINVAL, "tile smaller than a subdomain tile");
  DD_HIP(ddh::launch_packed_to_tiles(h->subs, h->nsub, h->nrhs, h->nfine, (const cplx<double>*)u, scale, tile, t,
                                     (hipStream_t)stream));
  return DD_OK;
}

dd_status dd_tile_descs(const dd_handle* h, dd_tile_desc* out) {
  DD_TRY(check_handle(h));
  if (!out) return fail(DD_EINVAL, "null argument");
  for (int j = 0; j < h->nsub; ++j) {
    const SubDesc& d = h->subs_h[j];
    out[j].nx = d.nx;
    out[j].ny = d.ny;
    out[j].edges = (d.i0 == d.ax ? 1 : 0) | (d.i0 + d.nx - 1 == d.bx ? 2 : 0) | (d.j0 == d.ay ? 4 : 0) |
                   (d.j0 + d.ny - 1 == d.by ? 8 : 0);
    out[j].robin = d.robin;
    out[j].kh = h->cs.kh;
  }
  return DD_OK;
}

dd_status dd_last_inner(const dd_handle* h, int32_t* iters, int32_t* flags, void* stream) {
  DD_TRY(check_handle(h));
  hipStream_t st = (hipStream_t)stream;
  const size_t cnt = (size_t)h->nsub * h->nrhs;
  if (iters) DD_HIP(hipMemcpyAsync(iters, h->iters, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
  if (flags) DD_HIP(hipMemcpyAsync(flags, h->flags, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

dd_status dd_outer_basis(dd_handle* h, int j, void* v, void* stream) {
  DD_TRY(check_handle(h));
  if (!v) return fail(DD_EINVAL, "null argument");
  if (j < 0 || j > h->restart) return fail(DD_EINVAL, "basis index out of range");
  const long long nd = h->ndof, vstr = (long long)(h->restart + 1) * nd;
  DD_HIP(hipMemcpy2DAsync(v, nd * sizeof(cplx<double>), h->Vo + (long long)j * nd, vstr * sizeof(cplx<double>),
                          nd * sizeof(cplx<double>), h->nrhs, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return DD_OK;
}

// ---- two-level method ---------------------------------------------------------------

int64_t dd_global_coarse_size(const dd_handle* h) { return (h && h->gc) ? h->gc->ncoarse : 0; }

dd_status dd_global_coarse_matrix(const dd_handle* h, double* out, double* min_pivot) {
  DD_TRY(check_handle(h));
  if (!h->gc) return fail(DD_EINVAL, "the handle has no global coarse space (coarse_intervals = 0)");
  if (!out) return fail(DD_EINVAL, "null argument");
  DD_HIP(hipMemcpy(out, h->gc->E0c, (size_t)h->gc->ncoarse * 9 * sizeof(double), hipMemcpyDeviceToHost));
  if (min_pivot) *min_pivot = h->gc->min_pivot;
  return DD_OK;
}

dd_status dd_op_global_restrict(dd_handle* h, const void* r, void* t, void* stream) {
  DD_TRY(check_handle(h));
  if (!h->gc) return fail(DD_EINVAL, "the handle has no global coarse space (coarse_intervals = 0)");
  if (!r || !t) return fail(DD_EINVAL, "null vector");
  hipStream_t st = (hipStream_t)stream;
  DD_HIP(h->gc->restrict_rhs((const cplx<double>*)r, h->ndof, nullptr, 0, nullptr, 1, st));
  DD_HIP(hipMemcpyAsync(t, h->gc->cv, (size_t)h->gc->ncoarse * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
  return DD_OK;
}

dd_status dd_op_global_coarse_solve(dd_handle* h, const void* t, void* y, void* stream) {
  DD_TRY(check_handle(h));
  if (!h->gc) return fail(DD_EINVAL, "the handle has no global coarse space (coarse_intervals = 0)");
  if (!t || !y) return fail(DD_EINVAL, "null vector");
  hipStream_t st = (hipStream_t)stream;
  const size_t nb = (size_t)h->gc->ncoarse * sizeof(cplx<double>);
  DD_HIP(hipMemcpyAsync(h->gc->cv, t, nb, hipMemcpyDeviceToDevice, st));
  DD_HIP(h->gc->solve(1, st));
  DD_HIP(hipMemcpyAsync(y, h->gc->cv + h->gc->ncoarse, nb, hipMemcpyDeviceToDevice, st));
  return DD_OK;
}

dd_status dd_op_global_correct(dd_handle* h, const void* r, const void* y, void* q, void* w, void* stream) {
  DD_TRY(check_handle(h));
  if (!h->gc) return fail(DD_EINVAL, "the handle has no global coarse space (coarse_intervals = 0)");
  if (!r || !y) return fail(DD_EINVAL, "null vector");
  hipStream_t st = (hipStream_t)stream;
  const size_t nb = (size_t)h->gc->ncoarse * sizeof(cplx<double>), nf = (size_t)h->ndof * sizeof(cplx<double>);
  DD_HIP(hipMemcpyAsync(h->gc->cv + h->gc->ncoarse, y, nb, hipMemcpyDeviceToDevice, st));
  DD_HIP(h->gc->correct((const cplx<double>*)r, h->ndof, nullptr, 0, nullptr, 1, st));
  if (q) DD_HIP(hipMemcpyAsync(q, h->gc->q, nf, hipMemcpyDeviceToDevice, st));
  if (w) DD_HIP(hipMemcpyAsync(w, h->gc->w, nf, hipMemcpyDeviceToDevice, st));
  return DD_OK;
}

}  // extern "C"
