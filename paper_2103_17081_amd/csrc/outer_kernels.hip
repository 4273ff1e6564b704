// FP64 kernels of the outer right-flexible FGMRES (Sec. 3) over the global system
// A u = f (Sec. 2, eq. 2), batched over independent right-hand sides that advance
// in lockstep; a right-hand side whose `done` flag is set is left untouched.
//
// Vectors: [nrhs][ndof] complex<double>, interior nodes x fastest.  Bases:
// basis(rhs, i) = base + (rhs * nvec + i) * ndof.
#include "kernels.hpp"
#include "outer.hpp"

namespace ddh {

// w = A v: the interior P1 stencil (centre 4 - kh2/2, E/W/N/S -1 - kh2/12,
// NE/SW -kh2/12), Dirichlet neighbours eliminated.
__global__ void __launch_bounds__(256) global_apply_kernel(Consts cs, const cplx<double>* __restrict__ v,
                                                            long long vstride, cplx<double>* __restrict__ w,
                                                            long long wstride, const int* __restrict__ done) {
  const int rhs = blockIdx.z;
  if (done && done[rhs]) return;
  const int m = cs.n - 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= m || j >= m) return;
  const double cc = 4.0 - cs.kh2 / 2.0, ce = -1.0 - cs.kh2 / 12.0, cd = -cs.kh2 / 12.0;
  const cplx<double>* x = v + rhs * vstride;
  const long long n = (long long)j * m + i;
  cplx<double> acc = cc * x[n];
  cplx<double> side = czero<double>();
  if (i > 0) side = side + x[n - 1];
  if (i < m - 1) side = side + x[n + 1];
  if (j > 0) side = side + x[n - m];
  if (j < m - 1) side = side + x[n + m];
  cplx<double> diag = czero<double>();
  if (i > 0 && j > 0) diag = diag + x[n - m - 1];
  if (i < m - 1 && j < m - 1) diag = diag + x[n + m + 1];
  acc = acc + ce * side + cd * diag;
  w[rhs * wstride + n] = acc;
}

hipError_t launch_global_apply(Consts cs, const cplx<double>* v, cplx<double>* w, int nrhs, hipStream_t st) {
  const long long nd = (long long)(cs.n - 1) * (cs.n - 1);
  return launch_global_apply_masked(cs, v, nd, w, nd, nrhs, nullptr, st);
}

hipError_t launch_global_apply_masked(Consts cs, const cplx<double>* v, long long vstride, cplx<double>* w,
                                      long long wstride, int nrhs, const int* done, hipStream_t st) {
  const int m = cs.n - 1;
  dim3 blk(64, 4);
  dim3 grd((m + 63) / 64, (m + 3) / 4, nrhs);
  hipLaunchKernelGGL(global_apply_kernel, grd, blk, 0, st, cs, v, vstride, w, wstride, done);
  return hipGetLastError();
}

// w = f - w (restart residual), per right-hand side strides.
__global__ void __launch_bounds__(256) residual_kernel(const cplx<double>* __restrict__ f, long long fstride,
                                                       cplx<double>* __restrict__ w, long long wstride,
                                                       long long ndof) {
  const int rhs = blockIdx.y;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < ndof;
       n += (long long)gridDim.x * blockDim.x)
    w[rhs * wstride + n] = f[rhs * fstride + n] - w[rhs * wstride + n];
}

hipError_t launch_residual(const cplx<double>* f, long long fstride, cplx<double>* w, long long wstride,
                           long long ndof, int nblk, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(residual_kernel, dim3(nblk, nrhs), dim3(256), 0, st, f, fstride, w, wstride, ndof);
  return hipGetLastError();
}

// part[rhs][blk][i] = sum over the block's rows of conj(basis_i) w for i < nvec,
// and, if with_norm, part[..][nvec] = sum |w|^2.
__global__ void __launch_bounds__(256) dots_kernel(const cplx<double>* __restrict__ basis, long long bstride,
                                                   const cplx<double>* __restrict__ w, long long wstride,
                                                   long long ndof, int nvec, int with_norm,
                                                   cplx<double>* __restrict__ part, int pstride,
                                                   const int* __restrict__ done) {
  const int rhs = blockIdx.y;
  if (done && done[rhs]) return;
  __shared__ cplx<double> red[4][kOuterMaxDots];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const long long chunk = (ndof + gridDim.x - 1) / gridDim.x;
  const long long n0 = blockIdx.x * chunk;
  const long long n1 = n0 + chunk < ndof ? n0 + chunk : ndof;
  const cplx<double>* x = w + rhs * wstride;
  const int nslots = nvec + (with_norm ? 1 : 0);
  for (int s0 = 0; s0 < nslots; s0 += kOuterMaxDots) {
    const int s1 = min(nslots, s0 + kOuterMaxDots);
    for (int s = s0; s < s1; ++s) {
      cplx<double> p = czero<double>();
      if (s < nvec) {
        const cplx<double>* b = basis + (rhs * bstride) + (long long)s * ndof;
        for (long long n = n0 + tid; n < n1; n += blockDim.x) p = p + cmulc(b[n], x[n]);
      } else {
        for (long long n = n0 + tid; n < n1; n += blockDim.x) p.re += cabs2(x[n]);
      }
      p.re = wave_sum(p.re);
      p.im = wave_sum(p.im);
      if (lane == 0) red[wave][s - s0] = p;
    }
    __syncthreads();
    for (int s = s0 + tid; s < s1; s += blockDim.x) {
      cplx<double> t = red[0][s - s0] + red[1][s - s0] + red[2][s - s0] + red[3][s - s0];
      part[((long long)rhs * gridDim.x + blockIdx.x) * pstride + s] = t;
    }
    __syncthreads();
  }
}

// out[rhs][s] = sum_blk part[rhs][blk][s]; mode 0: H[s] = out, 1: H[s] += out, 2: none.
__global__ void __launch_bounds__(256) reduce_parts_kernel(const cplx<double>* __restrict__ part, int nblk,
                                                           int pstride, int nslots, cplx<double>* __restrict__ out,
                                                           int ostride, cplx<double>* __restrict__ H, int hstride,
                                                           int mode, const int* __restrict__ done) {
  const int rhs = blockIdx.x;
  if (done && done[rhs]) return;
  for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
    cplx<double> acc = czero<double>();
    for (int b = 0; b < nblk; ++b) acc = acc + part[((long long)rhs * nblk + b) * pstride + s];
    out[rhs * ostride + s] = acc;
    if (H) {
      cplx<double>* hh = H + (long long)rhs * hstride + s;
      if (mode == 0) *hh = acc;
      else if (mode == 1) *hh = *hh + acc;
    }
  }
}

// w -= sum_i basis_i * coef[i], i < nvec.
__global__ void __launch_bounds__(256) update_kernel(const cplx<double>* __restrict__ basis, long long bstride,
                                                     cplx<double>* __restrict__ w, long long wstride,
                                                     long long ndof, int nvec,
                                                     const cplx<double>* __restrict__ coef, int cstride,
                                                     double sign, const int* __restrict__ done) {
  const int rhs = blockIdx.y;
  if (done && done[rhs]) return;
  __shared__ cplx<double> c[kOuterMaxDots];
  cplx<double>* x = w + rhs * wstride;
  for (int s0 = 0; s0 < nvec; s0 += kOuterMaxDots) {
    const int s1 = min(nvec, s0 + kOuterMaxDots);
    __syncthreads();
    for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x) c[s - s0] = coef[rhs * cstride + s];
    __syncthreads();
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < ndof;
         n += (long long)gridDim.x * blockDim.x) {
      cplx<double> acc = czero<double>();
      for (int s = s0; s < s1; ++s) acc = cfma(basis[rhs * bstride + (long long)s * ndof + n], c[s - s0], acc);
      x[n] = x[n] + sign * acc;
    }
  }
}

// out = w * (1 / scale[rhs]) with scale read from the device.
__global__ void __launch_bounds__(256) scale_kernel(const cplx<double>* w, long long wstride,
                                                    cplx<double>* out, long long ostride,
                                                    long long ndof, const double* __restrict__ scale,
                                                    const int* __restrict__ done) {
  const int rhs = blockIdx.y;
  if (done && done[rhs]) return;
  const double s = scale[rhs];
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < ndof;
       n += (long long)gridDim.x * blockDim.x)
    out[rhs * ostride + n] = inv * w[rhs * wstride + n];
}

// Givens step j of every active right-hand side (one thread each).
// H column j (j+1 entries) is in hcol; the norm^2 of the orthogonalised w in
// nrm2[rhs].  Applies the stored rotations, forms rotation j, updates g, stores the
// rotated column into R (column j), sets res[rhs] = |g_{j+1}| and done[rhs] when
// res <= atol[rhs], and hnext[rhs] = ||w||.
__global__ void givens_kernel(OuterState st, int j, int nrhs) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs || st.done[rhs]) return;
  const int m = st.restart;
  cplx<double>* col = st.H + (long long)rhs * (m + 1);
  const double hnext = sqrt(st.nrm2[rhs * st.nrm_stride].re);
  double* cs = st.cs + (long long)rhs * m;
  cplx<double>* sn = st.sn + (long long)rhs * m;
  cplx<double>* g = st.g + (long long)rhs * (m + 1);
  for (int i = 0; i < j; ++i) {
    const cplx<double> x0 = col[i], x1 = col[i + 1];
    col[i] = cs[i] * x0 + sn[i] * x1;
    col[i + 1] = cs[i] * x1 - cplx<double>{sn[i].re, -sn[i].im} * x0;
  }
  const cplx<double> av = col[j];
  const double aa = sqrt(cabs2(av));
  double c;
  cplx<double> s, r;
  if (hnext == 0.0) {
    c = 1.0; s = czero<double>(); r = av;
  } else if (aa == 0.0) {
    c = 0.0; s = cplx<double>{1.0, 0.0}; r = cplx<double>{hnext, 0.0};
  } else {
    const double t = hypot(aa, hnext);
    const cplx<double> ph{av.re / aa, av.im / aa};
    c = aa / t;
    s = (hnext / t) * ph;
    r = t * ph;
  }
  cs[j] = c;
  sn[j] = s;
  col[j] = r;
  cplx<double>* R = st.R + (long long)rhs * m * m;
  for (int i = 0; i <= j; ++i) R[(long long)j * m + i] = col[i];
  const cplx<double> gj = g[j];
  g[j + 1] = czero<double>() - cplx<double>{s.re, -s.im} * gj;
  g[j] = c * gj;
  const double res = sqrt(cabs2(g[j + 1]));
  st.res[rhs] = res;
  st.hnext[rhs] = hnext;
  st.steps[rhs] = j + 1;
  if (res <= st.atol[rhs] || hnext == 0.0) st.done[rhs] = 1;
}

// y = R^{-1} g over the first steps[rhs] columns (one thread per right-hand side).
__global__ void backsolve_kernel(OuterState st, int nrhs) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  const int m = st.restart;
  const int k = st.steps[rhs];
  const cplx<double>* R = st.R + (long long)rhs * m * m;
  const cplx<double>* g = st.g + (long long)rhs * (m + 1);
  cplx<double>* y = st.y + (long long)rhs * m;
  for (int i = k - 1; i >= 0; --i) {
    cplx<double> s = g[i];
    for (int jj = i + 1; jj < k; ++jj) s = s - R[(long long)jj * m + i] * y[jj];
    y[i] = s * cinv(R[(long long)i * m + i]);
  }
  for (int i = k; i < m; ++i) y[i] = czero<double>();
}

// Initialise a cycle: g = (beta, 0, ...), steps = 0, beta from the norm slot.
__global__ void cycle_init_kernel(OuterState st, int nrhs) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  const int m = st.restart;
  const double beta = sqrt(st.nrm2[rhs * st.nrm_stride].re);
  cplx<double>* g = st.g + (long long)rhs * (m + 1);
  for (int i = 0; i <= m; ++i) g[i] = czero<double>();
  g[0] = cplx<double>{beta, 0.0};
  st.hnext[rhs] = beta;
  st.res[rhs] = beta;
  st.steps[rhs] = 0;
  if (st.first_cycle) st.atol[rhs] = st.rtol * beta;
  st.done[rhs] = (beta <= st.atol[rhs]) ? 1 : 0;
}

hipError_t launch_dots(const cplx<double>* basis, long long bstride, const cplx<double>* w, long long wstride,
                       long long ndof, int nvec, int with_norm, cplx<double>* part, int pstride, int nblk,
                       int nrhs, const int* done, hipStream_t st) {
  hipLaunchKernelGGL(dots_kernel, dim3(nblk, nrhs), dim3(256), 0, st, basis, bstride, w, wstride, ndof, nvec,
                     with_norm, part, pstride, done);
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const cplx<double>* part, int nblk, int pstride, int nslots, cplx<double>* out,
                               int ostride, cplx<double>* H, int hstride, int mode, int nrhs, const int* done,
                               hipStream_t st) {
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(nrhs), dim3(256), 0, st, part, nblk, pstride, nslots, out,
                     ostride, H, hstride, mode, done);
  return hipGetLastError();
}

hipError_t launch_update(const cplx<double>* basis, long long bstride, cplx<double>* w, long long wstride,
                         long long ndof, int nvec, const cplx<double>* coef, int cstride, double sign, int nblk,
                         int nrhs, const int* done, hipStream_t st) {
  hipLaunchKernelGGL(update_kernel, dim3(nblk, nrhs), dim3(256), 0, st, basis, bstride, w, wstride, ndof, nvec,
                     coef, cstride, sign, done);
  return hipGetLastError();
}

hipError_t launch_scale(const cplx<double>* w, long long wstride, cplx<double>* out, long long ostride,
                        long long ndof, const double* scale, int nblk, int nrhs, const int* done,
                        hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel, dim3(nblk, nrhs), dim3(256), 0, st, w, wstride, out, ostride, ndof, scale,
                     done);
  return hipGetLastError();
}

hipError_t launch_givens(const OuterState& s, int j, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(givens_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, s, j, nrhs);
  return hipGetLastError();
}

hipError_t launch_backsolve(const OuterState& s, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(backsolve_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, s, nrhs);
  return hipGetLastError();
}

hipError_t launch_cycle_init(const OuterState& s, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(cycle_init_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, s, nrhs);
  return hipGetLastError();
}

}  // namespace ddh
