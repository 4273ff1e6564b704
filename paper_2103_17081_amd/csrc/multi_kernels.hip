// The plain form of the subdomain solves: the deflated GMRES of the batched kernel
// (Sec. 2, eq. 4: Krylov iteration on P B with P = I - B Z E^{-1} Z^T, started from P f,
// recovery u = x + Z E^{-1} Z^T (f - B x); classical Gram-Schmidt applied twice, Givens
// rotations), run as a sequence of batched launches per GMRES stage -- every launch covers
// all subdomains, one workgroup per subdomain -- with the iteration loop on the host, one
// host synchronisation per inner iteration and no graph.  FP64, one right-hand side.
//
// The stencil, restriction, coarse block solve and prolongation are the kernel-level
// operations on packed vectors; the kernels below carry the Krylov state of each solve
// in global memory.  The recovery's coarse vector is combined from the coarse solutions
// the iteration already formed: Z^T (f - B x) = Z^T f - sum_i y_i Z^T B v_i.
#include <algorithm>

#include "coarse.hpp"
#include "kernels.hpp"

namespace ddh {

namespace {

constexpr int kMT = 256;             // threads per workgroup
constexpr int kMW = kMT / kWave;     // waves per workgroup

__device__ __forceinline__ double wg_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kMW; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ bool skipped(const MultiArgs& a) { return a.done && *a.done; }

// f = R_j r / ||R_j r|| (the solve runs on the unit right-hand side and is rescaled at the
// end); every solve that is not skipped starts active.
__global__ void __launch_bounds__(kMT) mk_start_kernel(MultiArgs a) {
  __shared__ double red[kMW];
  const int s = blockIdx.x;
  const SubDesc d = a.subs[s];
  const int nj = d.nx * d.ny, ldg = a.cs.n - 1;
  const bool skip = skipped(a);
  const long long js = a.jdev ? (long long)*a.jdev : 0;
  const cplx<double>* r = a.r ? a.r + js * a.rslot : nullptr;
  cplx<double>* F = a.F + d.off;
  auto at = [&](int n) {
    if (!r) return F[n];
    const int lj = n / d.nx, li = n - lj * d.nx;
    return r[(long long)(d.j0 + lj - 1) * ldg + (d.i0 + li - 1)];
  };
  double p = 0.0;
  for (int n = threadIdx.x; n < nj; n += kMT) p += cabs2(at(n));
  const double fn = sqrt(wg_sum(p, red));
  const double sc = fn > 0.0 ? 1.0 / fn : 0.0;
  for (int n = threadIdx.x; n < nj; n += kMT) F[n] = sc * at(n);
  if (threadIdx.x == 0) {
    a.fnorm[s] = fn;
    a.active[s] = skip ? 0 : 1;
    a.notconv[s] = 0;
    a.iters[s] = 0;
  }
}

// out = x - y over all packed fine nodes (out may alias y).
__global__ void __launch_bounds__(kMT) mk_sub_kernel(const cplx<double>* x, const cplx<double>* y,
                                                      cplx<double>* out, long long n) {
  for (long long i = blockIdx.x * (long long)kMT + threadIdx.x; i < n; i += (long long)gridDim.x * kMT)
    out[i] = x[i] - y[i];
}

// beta = ||P f|| (the reference of the relative stopping test), g_0 = beta,
// v_0 = P f / beta; a solve with P f = 0 is done at once.
__global__ void __launch_bounds__(kMT) mk_init_kernel(MultiArgs a) {
  __shared__ double red[kMW];
  const int s = blockIdx.x;
  const SubDesc d = a.subs[s];
  const int nj = d.nx * d.ny, m1 = a.maxit + 1;
  const cplx<double>* w = a.W + d.off;
  double p = 0.0;
  for (int n = threadIdx.x; n < nj; n += kMT) p += cabs2(w[n]);
  const double beta = sqrt(wg_sum(p, red));
  if (beta > 0.0) {
    cplx<double>* V = a.V + d.off * (long long)m1;
    const double inv = 1.0 / beta;
    for (int n = threadIdx.x; n < nj; n += kMT) V[n] = inv * w[n];
  }
  if (threadIdx.x == 0) {
    a.ref[s] = beta;
    a.g[(long long)s * m1] = cplx<double>{beta, 0.0};
    if (!(beta > 0.0)) a.active[s] = 0;
  }
}

// Packed copy of basis vector k of every active solve (the stencil's input).
__global__ void __launch_bounds__(kMT) mk_basis_kernel(MultiArgs a, int k) {
  const int s = blockIdx.x;
  if (!a.active[s]) return;
  const SubDesc d = a.subs[s];
  const int nj = d.nx * d.ny;
  const cplx<double>* v = a.V + d.off * (long long)(a.maxit + 1) + (long long)k * nj;
  for (int n = threadIdx.x; n < nj; n += kMT) a.T[d.off + n] = v[n];
}

// One classical Gram-Schmidt pass on w = P B v_k: h = V_k^H w (accumulated into the
// Hessenberg column over the two passes), w -= V_k h.  The first pass also takes ||w||.
__global__ void __launch_bounds__(kMT) mk_gs_kernel(MultiArgs a, int k, int pass) {
  __shared__ double part[kMW][2 * (kMultiMaxIt + 1)];
  __shared__ cplx<double> hs[kMultiMaxIt + 1];
  const int s = blockIdx.x;
  if (!a.active[s]) return;
  const SubDesc d = a.subs[s];
  const int nj = d.nx * d.ny, m1 = a.maxit + 1;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const cplx<double>* V = a.V + d.off * (long long)m1;
  cplx<double>* w = a.W + d.off;
  for (int i = 0; i <= k; ++i) {
    cplx<double> p = czero<double>();
    for (int n = threadIdx.x; n < nj; n += kMT) p = p + cmulc(V[(long long)i * nj + n], w[n]);
    p.re = wave_sum(p.re);
    p.im = wave_sum(p.im);
    if (lane == 0) {
      part[wave][2 * i] = p.re;
      part[wave][2 * i + 1] = p.im;
    }
  }
  if (pass == 0) {
    double wn2 = 0.0;
    for (int n = threadIdx.x; n < nj; n += kMT) wn2 += cabs2(w[n]);
    wn2 = wave_sum(wn2);
    if (lane == 0) part[wave][2 * (k + 1)] = wn2;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= k + (pass == 0 ? 1 : 0); i += kMT) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int q = 0; q < kMW; ++q) {
      re += part[q][2 * i];
      if (i <= k) im += part[q][2 * i + 1];
    }
    if (i <= k) {
      hs[i] = cplx<double>{re, im};
      cplx<double>* H = a.H + (long long)s * m1;
      H[i] = pass == 0 ? hs[i] : H[i] + hs[i];
    } else {
      a.wn[s] = sqrt(re);
    }
  }
  __syncthreads();
  for (int n = threadIdx.x; n < nj; n += kMT) {
    cplx<double> x = w[n];
    for (int i = 0; i <= k; ++i) x = x - V[(long long)i * nj + n] * hs[i];
    w[n] = x;
  }
}

// h_{k+1,k} = ||w||; the earlier rotations applied to the Hessenberg column, the new
// rotation that annihilates h_{k+1,k}, the rotated right-hand side and the column of R;
// the residual estimate |g_{k+1}| against tol ||P f|| (or a breakdown); v_{k+1} = w / ||w||
// for solves that go on.
__global__ void __launch_bounds__(kMT) mk_givens_kernel(MultiArgs a, int k) {
  __shared__ double red[kMW];
  __shared__ int go;
  const int s = blockIdx.x;
  if (!a.active[s]) return;
  const SubDesc d = a.subs[s];
  const int nj = d.nx * d.ny, m1 = a.maxit + 1, m = a.maxit;
  const cplx<double>* w = a.W + d.off;
  double p = 0.0;
  for (int n = threadIdx.x; n < nj; n += kMT) p += cabs2(w[n]);
  const double hnext = sqrt(wg_sum(p, red));
  if (threadIdx.x == 0) {
    cplx<double>* col = a.H + (long long)s * m1;
    double* cs = a.csn + (long long)s * m;
    cplx<double>* sn = a.snn + (long long)s * m;
    cplx<double>* g = a.g + (long long)s * m1;
    for (int i = 0; i < k; ++i) {
      const cplx<double> x0 = col[i], x1 = col[i + 1];
      col[i] = cs[i] * x0 + sn[i] * x1;
      col[i + 1] = cs[i] * x1 - cplx<double>{sn[i].re, -sn[i].im} * x0;
    }
    const cplx<double> av = col[k];
    const double aa = sqrt(cabs2(av));
    double c;
    cplx<double> sv, rr;
    if (hnext == 0.0) {
      c = 1.0; sv = czero<double>(); rr = av;
    } else if (aa == 0.0) {
      c = 0.0; sv = cplx<double>{1.0, 0.0}; rr = cplx<double>{hnext, 0.0};
    } else {
      const double t = hypot(aa, hnext);
      const cplx<double> ph{av.re / aa, av.im / aa};
      c = aa / t;
      sv = (hnext / t) * ph;
      rr = t * ph;
    }
    cs[k] = c;
    sn[k] = sv;
    col[k] = rr;
    cplx<double>* R = a.R + (long long)s * m * m + (long long)k * m;
    for (int i = 0; i <= k; ++i) R[i] = col[i];
    const cplx<double> gk = g[k];
    g[k + 1] = czero<double>() - cplx<double>{sv.re, -sv.im} * gk;
    g[k] = c * gk;
    const double res = sqrt(cabs2(g[k + 1]));
    const bool conv = res <= a.tol * a.ref[s] || hnext <= 1e-14 * a.wn[s];
    a.iters[s] = k + 1;
    go = (!conv && k + 1 < a.maxit) ? 1 : 0;
    if (!go) a.active[s] = 0;
    if (!conv && !go) a.notconv[s] = 1;
  }
  __syncthreads();
  if (go) {
    cplx<double>* V = a.V + d.off * (long long)m1 + (long long)(k + 1) * nj;
    const double inv = 1.0 / hnext;
    for (int n = threadIdx.x; n < nj; n += kMT) V[n] = inv * w[n];
  }
}

__global__ void __launch_bounds__(kMT) mk_count_kernel(const int* __restrict__ active, int nsub,
                                                        int* __restrict__ out) {
  __shared__ int part[kMW];
  int mine = 0;
  for (int s = threadIdx.x; s < nsub; s += kMT) mine += active[s];
  mine = wave_sum(mine);
  if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    for (int w = 0; w < kMW; ++w) c += part[w];
    *out = c;
  }
}

// y = R^{-1} g; x = V y (packed X); the recovery's coarse vector
// c = E^{-1} Z^T f - sum_i y_i E^{-1} Z^T B v_i (packed Cv).
__global__ void __launch_bounds__(kMT) mk_final_kernel(MultiArgs a) {
  __shared__ cplx<double> y[kMultiMaxIt];
  const int s = blockIdx.x;
  const SubDesc d = a.subs[s];
  const int nj = d.nx * d.ny, m1 = a.maxit + 1, m = a.maxit;
  const int k = a.iters[s];
  if (threadIdx.x == 0) {
    const cplx<double>* R = a.R + (long long)s * m * m;
    const cplx<double>* g = a.g + (long long)s * m1;
    for (int i = k - 1; i >= 0; --i) {
      cplx<double> acc = g[i];
      for (int j = i + 1; j < k; ++j) acc = acc - R[(long long)j * m + i] * y[j];
      y[i] = acc * cinv(R[(long long)i * m + i]);
    }
  }
  __syncthreads();
  const cplx<double>* V = a.V + d.off * (long long)m1;
  for (int n = threadIdx.x; n < nj; n += kMT) {
    cplx<double> x = czero<double>();
    for (int i = 0; i < k; ++i) x = x + V[(long long)i * nj + n] * y[i];
    a.X[d.off + n] = x;
  }
  const int nc = d.mx * d.my;
  for (int e = threadIdx.x; e < nc; e += kMT) {
    cplx<double> c = a.Yk[d.coff + e];
    for (int i = 0; i < k; ++i) c = c - y[i] * a.Yk[(long long)(2 + i) * a.ncoarse + d.coff + e];
    a.Cv[d.coff + e] = c;
  }
}

// u = ||f|| (x + Z c): packed (all tile nodes) and at the owned nodes of z (plus zadd);
// iteration flags and counters.
__global__ void __launch_bounds__(kMT) mk_finish_kernel(MultiArgs a) {
  if (skipped(a)) return;
  const int s = blockIdx.x;
  const SubDesc d = a.subs[s];
  const int nj = d.nx * d.ny, ldg = a.cs.n - 1;
  const double fn = a.fnorm[s];
  if (a.U)
    for (int n = threadIdx.x; n < nj; n += kMT) a.U[d.off + n] = fn * (a.X[d.off + n] + a.Zc[d.off + n]);
  const int ow = d.oi1 - d.oi0 + 1, oh = d.oj1 - d.oj0 + 1;
  if (a.z) {
    const long long js = a.jdev ? (long long)*a.jdev : 0;
    cplx<double>* z = a.z + js * a.zslot;
    for (int n = threadIdx.x; n < ow * oh; n += kMT) {
      const int gj = d.oj0 + n / ow, gi = d.oi0 + n % ow;
      const long long loc = d.off + (long long)(gj - d.j0) * d.nx + (gi - d.i0);
      const long long gidx = (long long)(gj - 1) * ldg + (gi - 1);
      const cplx<double> u = fn * (a.X[loc] + a.Zc[loc]);
      z[gidx] = a.zadd ? u + a.zadd[gidx] : u;
    }
  }
  if (threadIdx.x == 0) {
    const int k = a.iters[s];
    if (a.flags) a.flags[s] = a.notconv[s] ? 2 : 0;
    if (a.counters) {
      const unsigned long long kk = (unsigned long long)k, nn = (unsigned long long)nj;
      const unsigned long long own = (unsigned long long)ow * oh, ncp = (unsigned long long)d.ncp;
      const unsigned long long fac_bytes = 16ull * (unsigned long long)coarse_solve_values(d);
      const unsigned long long bytes = 16ull * nn + (a.zadd ? 32ull : 16ull) * own + (kk + 1) * fac_bytes +
                                       16ull * ncp * (2 * kk + 2) + 16ull * nn * (2 * kk + 2 * kk * (kk + 1)) +
                                       32ull * nn;
      atomicAdd(a.counters + 0, kk);
      atomicAdd(a.counters + 1, 1ull);
      atomicMax(a.counters + 2, kk);
      atomicAdd(a.counters + 4, bytes);
    }
  }
}

}  // namespace

#define MK_TRY(x)                    \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

#define MK_LAUNCH(kernel, grid, ...)                                       \
  do {                                                                     \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kMT), 0, st, __VA_ARGS__); \
    MK_TRY(hipGetLastError());                                             \
  } while (0)

hipError_t run_multi_inner(const MultiArgs& a, int* active_host, hipStream_t st) {
  if (a.maxit < 1 || a.maxit > kMultiMaxIt) return hipErrorInvalidValue;
  const int ns = a.nsub;
  const long long nf = a.nfine;
  const unsigned fgrid = (unsigned)std::min<long long>((nf + kMT - 1) / kMT, 4096);
  MK_LAUNCH(mk_start_kernel, ns, a);
  // P f = f - B Z E^{-1} Z^T f, with E^{-1} Z^T f kept in coarse slot 0
  MK_TRY(launch_restrict(a.subs, ns, a.F, a.t, st));
  MK_TRY(launch_coarse_solve(a.subs, ns, a.fac, a.Ec, a.t, a.Yk, a.max_nc, st));
  MK_TRY(launch_prolong(a.subs, ns, a.Yk, a.T, st));
  MK_TRY(launch_local_apply<double>(a.subs, ns, a.cs, a.local_bc, a.T, a.Bv, a.max_nj, st));
  MK_LAUNCH(mk_sub_kernel, fgrid, (const cplx<double>*)a.F, (const cplx<double>*)a.Bv, a.W, nf);
  MK_LAUNCH(mk_init_kernel, ns, a);
  for (int k = 0; k < a.maxit; ++k) {
    MK_LAUNCH(mk_count_kernel, 1, (const int*)a.active, ns, a.nactive);
    MK_TRY(hipMemcpyAsync(active_host, a.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
    MK_TRY(hipStreamSynchronize(st));
    if (*active_host == 0) break;
    // w = P B v_k = B v_k - B Z E^{-1} Z^T B v_k, with E^{-1} Z^T B v_k kept in slot 2 + k.
    // (Stopped solves pass through the stencil and coarse launches on stale input; the
    // slots they fill beyond their own count are never read.)
    MK_LAUNCH(mk_basis_kernel, ns, a, k);
    MK_TRY(launch_local_apply<double>(a.subs, ns, a.cs, a.local_bc, a.T, a.Bv, a.max_nj, st));
    MK_TRY(launch_restrict(a.subs, ns, a.Bv, a.t, st));
    cplx<double>* yk = a.Yk + (long long)(2 + k) * a.ncoarse;
    MK_TRY(launch_coarse_solve(a.subs, ns, a.fac, a.Ec, a.t, yk, a.max_nc, st));
    MK_TRY(launch_prolong(a.subs, ns, yk, a.T, st));
    MK_TRY(launch_local_apply<double>(a.subs, ns, a.cs, a.local_bc, a.T, a.W, a.max_nj, st));
    MK_LAUNCH(mk_sub_kernel, fgrid, (const cplx<double>*)a.Bv, (const cplx<double>*)a.W, a.W, nf);
    MK_LAUNCH(mk_gs_kernel, ns, a, k, 0);
    MK_LAUNCH(mk_gs_kernel, ns, a, k, 1);
    MK_LAUNCH(mk_givens_kernel, ns, a, k);
  }
  // recovery and scatter
  MK_LAUNCH(mk_final_kernel, ns, a);
  MK_TRY(launch_prolong(a.subs, ns, a.Cv, a.Zc, st));
  MK_LAUNCH(mk_finish_kernel, ns, a);
  return hipSuccess;
}

}  // namespace ddh
