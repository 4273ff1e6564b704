// FP64 kernels of the outer right-flexible FGMRES (Sec. 3) over the global system
// A u = f (Sec. 2, eq. 2), batched over independent right-hand sides that advance
// in lockstep; a right-hand side whose `done` flag is set is left untouched.
//
// Vectors: [nrhs][ndof] complex<double>, interior nodes x fastest.  Bases:
// basis(rhs, i) = base + (rhs * nvec + i) * ndof.
#include <algorithm>

#include "kernels.hpp"
#include "outer.hpp"

namespace ddh {

// w = A v: the interior P1 stencil (centre 4 - kh2/2, E/W/N/S -1 - kh2/12,
// NE/SW -kh2/12), Dirichlet neighbours eliminated.
__global__ void __launch_bounds__(256) global_apply_kernel(Consts cs, const cplx<double>* __restrict__ v,
                                                            long long vstride, cplx<double>* __restrict__ w,
                                                            long long wstride, const int* __restrict__ done,
                                                            StepRef sr, long long vslot, long long wslot) {
  const int rhs = blockIdx.z;
  if (done && done[rhs]) return;
  const long long jj = sr.get();
  v += jj * vslot;
  w += jj * wslot;
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
                                      long long wstride, int nrhs, const int* done, hipStream_t st, StepRef sr,
                                      long long vslot, long long wslot) {
  const int m = cs.n - 1;
  dim3 blk(64, 4);
  dim3 grd((m + 63) / 64, (m + 3) / 4, nrhs);
  hipLaunchKernelGGL(global_apply_kernel, grd, blk, 0, st, cs, v, vstride, w, wstride, done, sr, vslot, wslot);
  return hipGetLastError();
}

// Advance the device-side outer step index (one thread).
__global__ void advance_step_kernel(int* jdev) {
  if (threadIdx.x == 0 && blockIdx.x == 0) jdev[0] += 1;
}

hipError_t launch_advance_step(int* jdev, hipStream_t st) {
  hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, st, jdev);
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

// Dot products of a tall-skinny basis with w, stage 1.  Block (chunk, group, rhs)
// covers kRowsPerThread * 256 consecutive rows and kVecsPerBlock consecutive slots:
// slot s < nvec is conj(basis_s) . w, slot nvec (if with_norm) is |w|^2.
// part layout: [rhs][slot][chunk].
constexpr int kRowsPerThread = 4;
constexpr int kVecsPerBlock = 8;
constexpr int kChunkRows = kRowsPerThread * 256;

__global__ void __launch_bounds__(256) dots_kernel(const cplx<double>* __restrict__ basis, long long bstride,
                                                   const cplx<double>* __restrict__ w, long long wstride,
                                                   long long ndof, int nvec, int with_norm,
                                                   cplx<double>* __restrict__ part, int pstride,
                                                   const int* __restrict__ done) {
  const int rhs = blockIdx.z;
  if (done && done[rhs]) return;
  __shared__ cplx<double> red[4][kVecsPerBlock];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int nchunk = gridDim.x;
  const long long n0 = (long long)blockIdx.x * kChunkRows + tid;
  const cplx<double>* x = w + rhs * wstride;
  cplx<double> xr[kRowsPerThread];
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const long long n = n0 + r * 256;
    xr[r] = n < ndof ? x[n] : czero<double>();
  }
  const int nslots = nvec + (with_norm ? 1 : 0);
  const int s0 = blockIdx.y * kVecsPerBlock;
  const int s1 = min(nslots, s0 + kVecsPerBlock);
  for (int s = s0; s < s1; ++s) {
    cplx<double> p = czero<double>();
    if (s < nvec) {
      const cplx<double>* b = basis + rhs * bstride + (long long)s * ndof;
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const long long n = n0 + r * 256;
        if (n < ndof) p = p + cmulc(b[n], xr[r]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) p.re += cabs2(xr[r]);
    }
    p.re = wave_sum(p.re);
    p.im = wave_sum(p.im);
    if (lane == 0) red[wave][s - s0] = p;
  }
  __syncthreads();
  for (int s = s0 + tid; s < s1; s += blockDim.x) {
    const cplx<double> t = red[0][s - s0] + red[1][s - s0] + red[2][s - s0] + red[3][s - s0];
    part[((long long)rhs * pstride + s) * nchunk + blockIdx.x] = t;
  }
}

// Delayed CGS2 pass 1: one sweep over the basis for two vectors.  Slots:
// [0, nvec): conj(V_i) . x1;  [nvec, 2 nvec): conj(V_i) . x2 (if x2);
// 2 nvec: |x1|^2;  2 nvec + 1: conj(x1) . x2;  2 nvec + 2: |x2|^2.
// Work items are (row chunk of kD2Chunk rows, group of kD2Vecs basis vectors); the
// last group also produces the three self slots.  Blocks take contiguous, chunk-major
// item ranges, so x1, x2 are loaded once per chunk change; the grid is fixed while
// nvec grows.  All loads of an item are issued before the products are formed, and
// each thread covers kD2Rows rows so the per-item reduction (DPP sums over 16-lane
// rows, then one LDS pass over the 16 row partials of the workgroup) is amortised over
// 128 KB of basis; the LDS partials alternate between two buffers, so an item needs one
// LDS-only barrier.  With `sr.jdev` set, nvec = *jdev and x1, x2 are basis vectors nvec
// and nvec+1 (graph-captured steps); otherwise nvec = sr.jhost and x1, x2 are the given
// vectors.  part layout: [rhs][chunk][slot] (pstride slots per chunk), dots2_chunks(ndof)
// chunks: an item's partials land in two or three contiguous runs (partials scattered
// one per slot row, 16 bytes apart by a chunk count, cost the sweep 8% of its time).
constexpr int kD2Rows = 8;
constexpr int kD2Vecs = 4;
constexpr int kD2Chunk = kD2Rows * 256;
constexpr int kD2Vals = 2 * (2 * kD2Vecs + 3);   // doubles reduced per item

__host__ __device__ int dots2_chunks(long long ndof) { return (int)((ndof + kD2Chunk - 1) / kD2Chunk); }

__global__ void __launch_bounds__(256) dots2_kernel(const cplx<double>* __restrict__ basis, long long bstride,
                                                    const cplx<double>* __restrict__ x1, long long x1stride,
                                                    const cplx<double>* __restrict__ x2, long long x2stride,
                                                    long long ndof, StepRef sr, int two_in,
                                                    cplx<double>* __restrict__ part, int pstride,
                                                    const int* __restrict__ done) {
  const int rhs = blockIdx.z;
  if (done && done[rhs]) return;
  __shared__ double red[2][16][kD2Vals];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int rowgrp = wave * 4 + lane / 16, li = lane % 16;
  const int nvec = sr.get();
  int buf = 0;
  const bool two = two_in != 0;
  const cplx<double>* X1 = sr.jdev ? basis + rhs * bstride + (long long)nvec * ndof : x1 + rhs * x1stride;
  const cplx<double>* X2 = sr.jdev ? basis + rhs * bstride + (long long)(nvec + 1) * ndof
                                   : (two ? x2 + rhs * x2stride : nullptr);
  const cplx<double>* Vb = basis + rhs * bstride;
  const int nchunk = dots2_chunks(ndof);
  const int ngroups = nvec > 0 ? (nvec + kD2Vecs - 1) / kD2Vecs : 1;
  const long long items = (long long)nchunk * ngroups;
  const long long lo = items * blockIdx.x / gridDim.x, hi = items * (blockIdx.x + 1) / gridDim.x;
  int cur = -1;
  cplx<double> a[kD2Rows], b[kD2Rows];
  for (long long item = lo; item < hi; ++item) {
    const int chunk = (int)(item / ngroups), group = (int)(item % ngroups);
    const long long n0 = (long long)chunk * kD2Chunk + tid;
    if (chunk != cur) {
      cur = chunk;
#pragma unroll
      for (int r = 0; r < kD2Rows; ++r) {
        const long long n = n0 + r * 256;
        a[r] = n < ndof ? X1[n] : czero<double>();
        b[r] = (two && n < ndof) ? X2[n] : czero<double>();
      }
    }
    const int s0 = group * kD2Vecs;
    const int s1 = min(nvec, s0 + kD2Vecs);
    const int cnt = s1 > s0 ? s1 - s0 : 0;
    cplx<double> v[kD2Vecs][kD2Rows];
#pragma unroll
    for (int q = 0; q < kD2Vecs; ++q) {
#pragma unroll
      for (int r = 0; r < kD2Rows; ++r) {
        const long long n = n0 + r * 256;
        v[q][r] = (q < cnt && n < ndof) ? load_stream(Vb + (long long)(s0 + q) * ndof + n) : czero<double>();
      }
    }
    double pv[kD2Vals];
#pragma unroll
    for (int q = 0; q < kD2Vecs; ++q) {
      cplx<double> p1 = czero<double>(), p2 = czero<double>();
#pragma unroll
      for (int r = 0; r < kD2Rows; ++r) {
        p1 = p1 + cmulc(v[q][r], a[r]);
        p2 = p2 + cmulc(v[q][r], b[r]);
      }
      pv[2 * q] = p1.re;
      pv[2 * q + 1] = p1.im;
      pv[2 * (kD2Vecs + q)] = p2.re;
      pv[2 * (kD2Vecs + q) + 1] = p2.im;
    }
    const bool self = group == ngroups - 1;
    {
      double s00 = 0.0, s22 = 0.0;
      cplx<double> s01 = czero<double>();
#pragma unroll
      for (int r = 0; r < kD2Rows; ++r) {
        s00 += cabs2(a[r]);
        s01 = s01 + cmulc(a[r], b[r]);
        s22 += cabs2(b[r]);
      }
      pv[4 * kD2Vecs] = s00;
      pv[4 * kD2Vecs + 1] = 0.0;
      pv[4 * kD2Vecs + 2] = s01.re;
      pv[4 * kD2Vecs + 3] = s01.im;
      pv[4 * kD2Vecs + 4] = s22;
      pv[4 * kD2Vecs + 5] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < kD2Vals; ++e) {
      const double t = row_sum<16>(pv[e]);
      if (li == 0) red[buf][rowgrp][e] = t;
    }
    // the readers below finish with red[buf] before this item's successor passes its own
    // barrier, so the item after that may overwrite it
    lds_barrier();
    if (tid < 2 * kD2Vecs + 3) {
      int slot = -1;
      if (tid < kD2Vecs) slot = tid < cnt ? s0 + tid : -1;
      else if (tid < 2 * kD2Vecs) slot = (two && tid - kD2Vecs < cnt) ? nvec + s0 + tid - kD2Vecs : -1;
      else slot = self ? 2 * nvec + (tid - 2 * kD2Vecs) : -1;
      if (slot >= 0) {
        cplx<double> t = czero<double>();
#pragma unroll
        for (int g = 0; g < 16; ++g) t = t + cplx<double>{red[buf][g][2 * tid], red[buf][g][2 * tid + 1]};
        part[((long long)rhs * nchunk + chunk) * pstride + slot] = t;
      }
    }
    buf ^= 1;
  }
}

// Sum of launch_dots2's partials over the row chunks, in two fixed-order stages so that
// the result does not depend on scheduling: stage 1 sums segments of kSegChunks chunks
// (seg[rhs][segment][slot]), stage 2 sums the segments into out[rhs][slot] for
// slot < mul * j + add.  Consecutive threads take consecutive slots (coalesced rows).
constexpr int kSegChunks = 8;
__host__ __device__ int dots2_segments(long long ndof) { return (dots2_chunks(ndof) + kSegChunks - 1) / kSegChunks; }

__global__ void __launch_bounds__(256) reduce_chunks_kernel(const cplx<double>* __restrict__ part, int nchunk,
                                                            int pstride, StepRef sr, int mul, int add,
                                                            cplx<double>* __restrict__ seg,
                                                            const int* __restrict__ done) {
  const int rhs = blockIdx.z;
  if (done && done[rhs]) return;
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= mul * sr.get() + add) return;
  const int nseg = (nchunk + kSegChunks - 1) / kSegChunks;
  const int c0 = blockIdx.y * kSegChunks, c1 = min(nchunk, c0 + kSegChunks);
  const cplx<double>* p = part + (long long)rhs * nchunk * pstride + s;
  cplx<double> v[kSegChunks];
#pragma unroll
  for (int q = 0; q < kSegChunks; ++q) v[q] = c0 + q < c1 ? p[(long long)(c0 + q) * pstride] : czero<double>();
  cplx<double> acc = czero<double>();
#pragma unroll
  for (int q = 0; q < kSegChunks; ++q) acc = acc + v[q];
  seg[((long long)rhs * nseg + blockIdx.y) * pstride + s] = acc;
}

__global__ void __launch_bounds__(256) reduce_segments_kernel(const cplx<double>* __restrict__ seg, int nseg,
                                                              int pstride, StepRef sr, int mul, int add,
                                                              cplx<double>* __restrict__ out, int ostride,
                                                              const int* __restrict__ done) {
  const int rhs = blockIdx.z;
  if (done && done[rhs]) return;
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= mul * sr.get() + add) return;
  const cplx<double>* p = seg + (long long)rhs * nseg * pstride + s;
  cplx<double> acc = czero<double>();
  for (int g0 = 0; g0 < nseg; g0 += kSegChunks) {
    // a batch of independent loads, then the sums in segment order
    cplx<double> v[kSegChunks];
#pragma unroll
    for (int q = 0; q < kSegChunks; ++q) v[q] = g0 + q < nseg ? p[(long long)(g0 + q) * pstride] : czero<double>();
#pragma unroll
    for (int q = 0; q < kSegChunks; ++q) acc = acc + v[q];
  }
  out[(long long)rhs * ostride + s] = acc;
}

// Stage 2: out[rhs][s] = sum over chunks for s < nslots = mul * j + add (j from the
// StepRef); mode 0: H[s] = out, 1: H[s] += out, 2: none.  One wavefront per slot,
// striding over the slots.
__global__ void __launch_bounds__(64) reduce_parts_kernel(const cplx<double>* __restrict__ part, int nchunk,
                                                          int pstride, StepRef sr, int mul, int add,
                                                          cplx<double>* __restrict__ out, int ostride,
                                                          cplx<double>* __restrict__ H, int hstride, int mode,
                                                          const int* __restrict__ done) {
  const int rhs = blockIdx.y;
  if (done && done[rhs]) return;
  const int nslots = mul * sr.get() + add;
  for (int s = blockIdx.x; s < nslots; s += gridDim.x) {
    const cplx<double>* p = part + ((long long)rhs * pstride + s) * nchunk;
    cplx<double> acc = czero<double>();
    for (int c = threadIdx.x; c < nchunk; c += 64) acc = acc + p[c];
    acc.re = wave_sum(acc.re);
    acc.im = wave_sum(acc.im);
    if (threadIdx.x == 0) {
      out[rhs * ostride + s] = acc;
      if (H) {
        cplx<double>* hh = H + (long long)rhs * hstride + s;
        if (mode == 0) *hh = acc;
        else if (mode == 1) *hh = *hh + acc;
      }
    }
  }
}

// w += sign * sum_i basis_i * coef[i], i < nvec.  Each thread owns kRowsPerThread rows
// (strided by 256 inside a chunk) and keeps independent accumulators.
__global__ void __launch_bounds__(256) update_kernel(const cplx<double>* __restrict__ basis, long long bstride,
                                                     cplx<double>* __restrict__ w, long long wstride,
                                                     long long ndof, int nvec,
                                                     const cplx<double>* __restrict__ coef, int cstride,
                                                     double sign, const int* __restrict__ done) {
  const int rhs = blockIdx.y;
  if (done && done[rhs]) return;
  __shared__ cplx<double> c[kOuterMaxDots];
  cplx<double>* x = w + rhs * wstride;
  const long long n0 = (long long)blockIdx.x * kChunkRows + threadIdx.x;
  cplx<double> acc[kRowsPerThread];
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) acc[r] = czero<double>();
  for (int s0 = 0; s0 < nvec; s0 += kOuterMaxDots) {
    const int s1 = min(nvec, s0 + kOuterMaxDots);
    __syncthreads();
    for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x) c[s - s0] = coef[rhs * cstride + s];
    __syncthreads();
    for (int q0 = s0; q0 < s1; q0 += kVecsPerBlock) {
      cplx<double> vv[kVecsPerBlock][kRowsPerThread];
#pragma unroll
      for (int q = 0; q < kVecsPerBlock; ++q) {
#pragma unroll
        for (int r = 0; r < kRowsPerThread; ++r) {
          const long long n = n0 + r * 256;
          vv[q][r] = (q0 + q < s1 && n < ndof) ? basis[rhs * bstride + (long long)(q0 + q) * ndof + n]
                                                : czero<double>();
        }
      }
#pragma unroll
      for (int q = 0; q < kVecsPerBlock; ++q) {
        if (q0 + q < s1) {
          const cplx<double> cs = c[q0 + q - s0];
#pragma unroll
          for (int r = 0; r < kRowsPerThread; ++r) acc[r] = cfma(vv[q][r], cs, acc[r]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const long long n = n0 + r * 256;
    if (n < ndof) x[n] = x[n] + sign * acc[r];
  }
}

// The update sweep runs 512-thread workgroups over chunks of 2048 rows (4 per thread): at
// the large workload's shape this streams 7.1 TB/s against 6.5 TB/s for 256 threads over
// 1024 rows, and chunks of 1536 or 3072 rows are slower still (4.9, 5.9 TB/s).
constexpr int kUpdThreads = 512;
constexpr int kUpdChunkRows = kRowsPerThread * kUpdThreads;

// Delayed CGS2 pass 2 (one sweep over the basis V_j for two outputs):
//   v_j     = u~_j / alpha - V_j (s / alpha)                     (slot j, in place)
//   u~_{j+1} = (w - V_j (c - s h_jj / alpha) - u~_j h_jj / alpha) / gamma_{j+1}
//                                                                 (slot j+1, in place of w)
// coefficient vectors a = s / alpha and b = c - s h_jj / alpha and the scalars
// (1/alpha, h_jj/alpha, 1/gamma) come from dcgs2_step_kernel.
__global__ void __launch_bounds__(kUpdThreads) dcgs2_update_kernel(cplx<double>* __restrict__ basis, long long bstride,
                                                           long long ndof, StepRef sr,
                                                           const cplx<double>* __restrict__ ca,
                                                           const cplx<double>* __restrict__ cb, int cstride,
                                                           const cplx<double>* __restrict__ scal,
                                                           const int* __restrict__ done) {
  const int rhs = blockIdx.y;
  if (done && done[rhs]) return;
  const int j = sr.get();
  __shared__ cplx<double> la[kOuterMaxDots], lb[kOuterMaxDots];
  cplx<double>* V = basis + rhs * bstride;
  const long long n0 = (long long)blockIdx.x * kUpdChunkRows + threadIdx.x;
  cplx<double> acc_a[kRowsPerThread], acc_b[kRowsPerThread];
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) { acc_a[r] = czero<double>(); acc_b[r] = czero<double>(); }
  for (int s0 = 0; s0 < j; s0 += kOuterMaxDots) {
    const int s1 = min(j, s0 + kOuterMaxDots);
    __syncthreads();
    for (int q = s0 + threadIdx.x; q < s1; q += blockDim.x) {
      la[q - s0] = ca[rhs * cstride + q];
      lb[q - s0] = cb[rhs * cstride + q];
    }
    __syncthreads();
    // batches of kVecsPerBlock basis vectors: all loads of a batch are issued first
    for (int q0 = s0; q0 < s1; q0 += kVecsPerBlock) {
      cplx<double> vv[kVecsPerBlock][kRowsPerThread];
#pragma unroll
      for (int q = 0; q < kVecsPerBlock; ++q) {
#pragma unroll
        for (int r = 0; r < kRowsPerThread; ++r) {
          const long long n = n0 + r * kUpdThreads;
          vv[q][r] = (q0 + q < s1 && n < ndof) ? load_stream(V + (long long)(q0 + q) * ndof + n) : czero<double>();
        }
      }
#pragma unroll
      for (int q = 0; q < kVecsPerBlock; ++q) {
        if (q0 + q < s1) {
          const cplx<double> xa = la[q0 + q - s0], xb = lb[q0 + q - s0];
#pragma unroll
          for (int r = 0; r < kRowsPerThread; ++r) {
            acc_a[r] = cfma(vv[q][r], xa, acc_a[r]);
            acc_b[r] = cfma(vv[q][r], xb, acc_b[r]);
          }
        }
      }
    }
  }
  const cplx<double> inv_alpha = scal[rhs * 4 + 0], e = scal[rhs * 4 + 1], inv_gamma = scal[rhs * 4 + 2];
  cplx<double>* uj = V + (long long)j * ndof;
  cplx<double>* w = V + (long long)(j + 1) * ndof;
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const long long n = n0 + r * kUpdThreads;
    if (n < ndof) {
      const cplx<double> uo = uj[n];
      uj[n] = inv_alpha.re * uo - acc_a[r];
      w[n] = inv_gamma.re * (w[n] - acc_b[r] - uo * e);
    }
  }
}

// Rotations 0..jc-1 applied to the column lcol[0..jc] by all threads of a 256-thread
// workgroup.  Rotation i maps (x_i, col_{i+1}) to the rotated entry
// c_i x_i + s_i col_{i+1} and the carried entry x_{i+1} = c_i col_{i+1} - conj(s_i) x_i,
// with x_0 = col_0; the rotated column is (entries 0..jc-1, x_jc).  The carried entry
// obeys the affine recurrence x_{i+1} = a_i + m_i x_i (a_i = c_i col_{i+1},
// m_i = -conj(s_i), |m_i| <= 1), so each thread composes the maps of a segment of
// rotations, a scan over the threads composes the segments (shuffles within a wave,
// the four wave totals through `wmap`), and each thread then replays its segment from
// its starting value: depth about 2 jc / 256 + 8 instead of jc.
__device__ __forceinline__ cplx<double> cshfl_up(cplx<double> v, int o) {
  return cplx<double>{__shfl_up(v.re, o, kWave), __shfl_up(v.im, o, kWave)};
}

__device__ void rotate_column_scan(cplx<double>* lcol, const double* lcs, const cplx<double>* lsn, int jc,
                                   cplx<double>* wmap) {
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int seg = (jc + 255) / 256;
  const int i0 = min(tid * seg, jc), i1 = min(i0 + seg, jc);
  const cplx<double> one{1.0, 0.0};
  const cplx<double> xstart = lcol[0];
  const cplx<double> xend = i1 > i0 ? lcol[i1] : czero<double>();
  // this segment's map x -> A + M x
  cplx<double> A = czero<double>(), M = one;
  for (int i = i0; i < i1; ++i) {
    const cplx<double> m{-lsn[i].re, lsn[i].im};
    const cplx<double> a = lcs[i] * (i + 1 < i1 ? lcol[i + 1] : xend);
    A = a + m * A;
    M = m * M;
  }
  // inclusive scan within the wave: (A, M) <- (A, M) o (maps of the lanes below)
  for (int o = 1; o < kWave; o <<= 1) {
    const cplx<double> pA = cshfl_up(A, o), pM = cshfl_up(M, o);
    if (lane >= o) {
      A = A + M * pA;
      M = M * pM;
    }
  }
  cplx<double> eA = cshfl_up(A, 1), eM = cshfl_up(M, 1);   // through the previous lane
  if (lane == 0) {
    eA = czero<double>();
    eM = one;
  }
  if (lane == kWave - 1) {
    wmap[2 * wave] = A;
    wmap[2 * wave + 1] = M;
  }
  __syncthreads();
  // composition of the earlier waves, then the entry carried into this segment
  cplx<double> PA = czero<double>(), PM = one;
  for (int w = 0; w < wave; ++w) {
    const cplx<double> WA = wmap[2 * w], WM = wmap[2 * w + 1];
    PA = WA + WM * PA;
    PM = WM * PM;
  }
  cplx<double> x = eA + eM * (PA + PM * xstart);
  // replay the segment; entry i1 (the next segment's first) was read before the barrier
  for (int i = i0; i < i1; ++i) {
    const cplx<double> x1 = i + 1 < i1 ? lcol[i + 1] : xend;
    const double c = lcs[i];
    const cplx<double> sv = lsn[i];
    lcol[i] = c * x + sv * x1;
    x = c * x1 - cplx<double>{sv.re, -sv.im} * x;
  }
  if (i1 == jc && i1 > i0) lcol[jc] = x;
}

// Delayed CGS2 bookkeeping of step j for every active right-hand side (one workgroup
// each).  From the pass-1 dots (s = V_j^H u~_j, c = V_j^H w, nu = |u~_j|^2,
// mu = u~_j^H w, ww = |w|^2):
//   alpha = sqrt(nu - |s|^2)  (norm of u~_j after reorthogonalisation);
//   column j-1 becomes final: h_{i,j-1} = t_i + gamma_j s_i (i < j, t = the tentative
//   column kept from step j-1), h_{j,j-1} = gamma_j alpha; it is rotated into R
//   and the residual estimate |g_j| decides convergence (with j columns);
//   tentative column j: t_i = c_i (i < j), t_j = h_jj = (mu - s^H c) / alpha;
//   gamma_{j+1} = sqrt(ww - |c|^2 - |h_jj|^2) (Pythagoras; only a scaling that the next
//   step corrects exactly through nu).
// Step 0 has no column to finalise; it sets g_0 = beta * alpha.
__global__ void __launch_bounds__(256) dcgs2_step_kernel(OuterState st, StepRef sr, long long ndof,
                                                         const cplx<double>* __restrict__ dots, int dstride, int has_w,
                                                         cplx<double>* __restrict__ ca, cplx<double>* __restrict__ cb,
                                                         int cstride, cplx<double>* __restrict__ scal) {
  const int rhs = blockIdx.x;
  if (st.done[rhs]) return;
  const int j = sr.get();
  if (threadIdx.x == 0 && has_w) {
    // one preconditioner application and the two basis sweeps of this step
    st.applies[rhs] += 1;
    atomicAdd(st.sweep_bytes + 0, 16ull * (unsigned long long)ndof * (unsigned long long)(j + 2));
    atomicAdd(st.sweep_bytes + 1, 16ull * (unsigned long long)ndof * (unsigned long long)(j + 4));
  }
  extern __shared__ __align__(16) unsigned char gsm[];
  const int m = st.restart;
  cplx<double>* lcol = (cplx<double>*)gsm;          // j + 1 entries
  cplx<double>* lsn = lcol + (j + 2);
  double* lcs = (double*)(lsn + (j + 1));
  __shared__ double red[4];
  __shared__ cplx<double> redc[4];
  __shared__ double sh_alpha;
  __shared__ int sh_conv;
  __shared__ cplx<double> wmap[8];
  const cplx<double>* D = dots + (long long)rhs * dstride;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  // |s|^2
  double ss = 0.0;
  for (int i = tid; i < j; i += blockDim.x) ss += cabs2(D[i]);
  ss = wave_sum(ss);
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  if (tid == 0) {
    const double nu = D[2 * j].re;
    const double a2 = nu - (red[0] + red[1] + red[2] + red[3]);
    sh_alpha = sqrt(a2 > 1e-300 ? a2 : 1e-300);
    sh_conv = 0;
  }
  __syncthreads();
  const double alpha = sh_alpha;
  cplx<double>* T = st.H + (long long)rhs * (m + 1);   // tentative column
  const double gamma = st.hnext[rhs];                   // gamma_j from step j-1
  cplx<double>* g = st.g + (long long)rhs * (m + 1);
  if (j == 0) {
    if (tid == 0) g[0] = cplx<double>{g[0].re * alpha, g[0].im * alpha};
  } else {
    // finalise column jc = j-1 and rotate it
    const int jc = j - 1;
    double* cs = st.cs + (long long)rhs * m;
    cplx<double>* sn = st.sn + (long long)rhs * m;
    for (int i = tid; i <= jc; i += blockDim.x) {
      lcol[i] = T[i] + gamma * D[i];
      if (i < jc) { lsn[i] = sn[i]; lcs[i] = cs[i]; }
    }
    __syncthreads();
    rotate_column_scan(lcol, lcs, lsn, jc, wmap);
    __syncthreads();
    if (tid == 0) {
      const double hnext = gamma * alpha;
      const cplx<double> av = lcol[jc];
      const double aa = sqrt(cabs2(av));
      double c;
      cplx<double> sv, r;
      if (hnext == 0.0) {
        c = 1.0; sv = czero<double>(); r = av;
      } else if (aa == 0.0) {
        c = 0.0; sv = cplx<double>{1.0, 0.0}; r = cplx<double>{hnext, 0.0};
      } else {
        const double t = hypot(aa, hnext);
        const cplx<double> ph{av.re / aa, av.im / aa};
        c = aa / t;
        sv = (hnext / t) * ph;
        r = t * ph;
      }
      cs[jc] = c;
      sn[jc] = sv;
      lcol[jc] = r;
      const cplx<double> gj = g[jc];
      g[jc + 1] = czero<double>() - cplx<double>{sv.re, -sv.im} * gj;
      g[jc] = c * gj;
      const double res = sqrt(cabs2(g[jc + 1]));
      st.res[rhs] = res;
      st.steps[rhs] = j;
      sh_conv = (res <= st.atol[rhs] || hnext == 0.0) ? 1 : 0;
    }
    __syncthreads();
    cplx<double>* R = st.R + (long long)rhs * m * m + (long long)jc * m;
    for (int i = tid; i <= jc; i += blockDim.x) R[i] = lcol[i];
  }
  if (sh_conv || !has_w) {
    if (tid == 0 && sh_conv) st.done[rhs] = 1;
    return;
  }
  // tentative column j and the pass-2 coefficients
  cplx<double> sc = czero<double>();
  double cc = 0.0;
  for (int i = tid; i < j; i += blockDim.x) {
    sc = sc + cmulc(D[i], D[j + i]);
    cc += cabs2(D[j + i]);
  }
  sc.re = wave_sum(sc.re); sc.im = wave_sum(sc.im); cc = wave_sum(cc);
  __syncthreads();
  if (lane == 0) { redc[wave] = sc; red[wave] = cc; }
  __syncthreads();
  const cplx<double> sTc = redc[0] + redc[1] + redc[2] + redc[3];
  const double csum = red[0] + red[1] + red[2] + red[3];
  const cplx<double> mu = D[2 * j + 1];
  const double ww = D[2 * j + 2].re;
  const cplx<double> hjj = (1.0 / alpha) * (mu - sTc);
  const cplx<double> e = (1.0 / alpha) * hjj;
  for (int i = tid; i < j; i += blockDim.x) {
    const cplx<double> si = D[i], ci = D[j + i];
    T[i] = ci;
    ca[rhs * cstride + i] = (1.0 / alpha) * si;
    cb[rhs * cstride + i] = ci - si * e;
  }
  if (tid == 0) {
    T[j] = hjj;
    double g2 = ww - csum - cabs2(hjj);
    const double floor2 = 1e-28 * (ww > 0 ? ww : 1.0);
    if (!(g2 > floor2)) g2 = floor2;
    const double gam = sqrt(g2);
    st.hnext[rhs] = gam;
    scal[rhs * 4 + 0] = cplx<double>{1.0 / alpha, 0.0};
    scal[rhs * 4 + 1] = e;
    scal[rhs * 4 + 2] = cplx<double>{1.0 / gam, 0.0};
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

constexpr int kGivensMax = 4000;   // longest outer cycle the bookkeeping stages in LDS

// y = R^{-1} g over the first steps[rhs] columns (one workgroup per right-hand side,
// column-oriented back substitution: after y_i is known every thread updates its rows).
__global__ void __launch_bounds__(256) backsolve_kernel(OuterState st) {
  const int rhs = blockIdx.x;
  const int m = st.restart;
  const int k = st.steps[rhs];
  const cplx<double>* R = st.R + (long long)rhs * m * m;
  cplx<double>* g = st.g + (long long)rhs * (m + 1);
  cplx<double>* y = st.y + (long long)rhs * m;
  __shared__ cplx<double> yi;
  for (int i = k - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      yi = g[i] * cinv(R[(long long)i * m + i]);
      y[i] = yi;
    }
    __syncthreads();
    const cplx<double> v = yi;
    for (int l = threadIdx.x; l < i; l += blockDim.x) g[l] = g[l] - R[(long long)i * m + l] * v;
    __syncthreads();
  }
  for (int i = k + threadIdx.x; i < m; i += blockDim.x) y[i] = czero<double>();
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

int outer_chunks(long long ndof) { return (int)((ndof + kChunkRows - 1) / kChunkRows); }

// Deterministic pseudo-random fill (a 64-bit mix of the index and seed mapped to
// [-1, 1)), used only to give the autotuner representative data.
__global__ void fill_hash_kernel(cplx<double>* __restrict__ x, long long n, unsigned long long seed) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ull + seed;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = cplx<double>{(double)(z & 0xffffffffull) / 2147483648.0 - 1.0, (double)(z >> 32) / 2147483648.0 - 1.0};
  }
}

hipError_t launch_fill_hash(cplx<double>* x, long long n, unsigned long long seed, hipStream_t st) {
  hipLaunchKernelGGL(fill_hash_kernel, dim3(2048), dim3(256), 0, st, x, n, seed);
  return hipGetLastError();
}

hipError_t configure_outer() {
  const int lds = (int)((size_t)(kGivensMax + 2) * 40);
  return hipFuncSetAttribute((const void*)dcgs2_step_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}


constexpr int kMaxSweepBlocks = 4096;   // grid cap of the striding outer sweeps

hipError_t launch_dots(const cplx<double>* basis, long long bstride, const cplx<double>* w, long long wstride,
                       long long ndof, int nvec, int with_norm, cplx<double>* part, int pstride, int nrhs,
                       const int* done, hipStream_t st) {
  const int nslots = nvec + (with_norm ? 1 : 0);
  dim3 grid(outer_chunks(ndof), (nslots + kVecsPerBlock - 1) / kVecsPerBlock, nrhs);
  hipLaunchKernelGGL(dots_kernel, grid, dim3(256), 0, st, basis, bstride, w, wstride, ndof, nvec, with_norm,
                     part, pstride, done);
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const cplx<double>* part, int nchunk, int pstride, StepRef sr, int mul, int add,
                               int jmax, cplx<double>* out, int ostride, cplx<double>* H, int hstride, int mode,
                               int nrhs, const int* done, hipStream_t st) {
  const int grid = std::min(mul * jmax + add, 1024);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid, nrhs), dim3(64), 0, st, part, nchunk, pstride, sr,
                     mul, add, out, ostride, H, hstride, mode, done);
  return hipGetLastError();
}

hipError_t launch_update(const cplx<double>* basis, long long bstride, cplx<double>* w, long long wstride,
                         long long ndof, int nvec, const cplx<double>* coef, int cstride, double sign, int nrhs,
                         const int* done, hipStream_t st) {
  hipLaunchKernelGGL(update_kernel, dim3(outer_chunks(ndof), nrhs), dim3(256), 0, st, basis, bstride, w, wstride,
                     ndof, nvec, coef, cstride, sign, done);
  return hipGetLastError();
}

hipError_t launch_scale(const cplx<double>* w, long long wstride, cplx<double>* out, long long ostride,
                        long long ndof, const double* scale, int nblk, int nrhs, const int* done,
                        hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel, dim3(nblk, nrhs), dim3(256), 0, st, w, wstride, out, ostride, ndof, scale,
                     done);
  return hipGetLastError();
}

hipError_t launch_reduce_chunks(const cplx<double>* part, long long ndof, int pstride, StepRef sr, int mul, int add,
                                int jmax, cplx<double>* out, int ostride, int nrhs, const int* done, hipStream_t st) {
  const int nchunk = dots2_chunks(ndof), nseg = dots2_segments(ndof);
  const int sblocks = (mul * jmax + add + 255) / 256;
  // the segment sums go after the partials of every right-hand side
  cplx<double>* seg = const_cast<cplx<double>*>(part) + (long long)nrhs * nchunk * pstride;
  hipLaunchKernelGGL(reduce_chunks_kernel, dim3(sblocks, nseg, nrhs), dim3(256), 0, st, part, nchunk, pstride, sr,
                     mul, add, seg, done);
  hipLaunchKernelGGL(reduce_segments_kernel, dim3(sblocks, 1, nrhs), dim3(256), 0, st, (const cplx<double>*)seg, nseg,
                     pstride, sr, mul, add, out, ostride, done);
  return hipGetLastError();
}

hipError_t launch_dots2(const cplx<double>* basis, long long bstride, const cplx<double>* x1, long long x1stride,
                        const cplx<double>* x2, long long x2stride, long long ndof, StepRef sr, int two, int jmax,
                        cplx<double>* part, int pstride, int nrhs, const int* done, hipStream_t st, int max_blocks) {
  const int groups = jmax > 0 ? (jmax + kD2Vecs - 1) / kD2Vecs : 1;
  const long long items = (long long)dots2_chunks(ndof) * groups;
  const int grid = (int)std::min<long long>(items, max_blocks > 0 ? max_blocks : kMaxSweepBlocks);
  // (each workgroup takes a contiguous range of about items / grid items)
  hipLaunchKernelGGL(dots2_kernel, dim3(grid, 1, nrhs), dim3(256), 0, st, basis, bstride, x1, x1stride, x2, x2stride,
                     ndof, sr, two, part, pstride, done);
  return hipGetLastError();
}

hipError_t launch_dcgs2_step(const OuterState& s, StepRef sr, int jmax, long long ndof, const cplx<double>* dots,
                             int dstride, int has_w, cplx<double>* ca, cplx<double>* cb, int cstride,
                             cplx<double>* scal, int nrhs, hipStream_t st) {
  if (jmax > kGivensMax) return hipErrorInvalidValue;
  const size_t lds =
      (size_t)(jmax + 2) * sizeof(cplx<double>) + (size_t)(jmax + 1) * (sizeof(cplx<double>) + sizeof(double));
  hipLaunchKernelGGL(dcgs2_step_kernel, dim3(nrhs), dim3(256), lds, st, s, sr, ndof, dots, dstride, has_w, ca, cb,
                     cstride, scal);
  return hipGetLastError();
}

hipError_t launch_dcgs2_update(cplx<double>* basis, long long bstride, long long ndof, StepRef sr,
                               const cplx<double>* ca, const cplx<double>* cb, int cstride, const cplx<double>* scal,
                               int nrhs, const int* done, hipStream_t st) {
  const int grid = (int)((ndof + kUpdChunkRows - 1) / kUpdChunkRows);
  hipLaunchKernelGGL(dcgs2_update_kernel, dim3(grid, nrhs), dim3(kUpdThreads), 0, st, basis, bstride, ndof, sr,
                     ca, cb, cstride, scal, done);
  return hipGetLastError();
}


hipError_t launch_backsolve(const OuterState& s, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(backsolve_kernel, dim3(nrhs), dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_cycle_init(const OuterState& s, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(cycle_init_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, s, nrhs);
  return hipGetLastError();
}

}  // namespace ddh
