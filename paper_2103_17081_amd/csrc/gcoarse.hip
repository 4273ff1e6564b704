// Global coarse space of the two-level method: Z_0, E_0 = Z_0^T A Z_0, its block
// cyclic reduction and the coarse correction (definitions in gcoarse.hpp).
//
// The global matrix A has homogeneous Dirichlet conditions on the boundary of the
// unit square (Sec. 2, eqs. 1-2), so it is real; Z_0 is real, hence E_0 and all of its
// factors are real FP64 and only the vectors are complex.
#include "gcoarse.hpp"

#include <algorithm>
#include <cmath>

namespace ddh {

namespace {

// Hat of coarse line c (0..M) at fine index i; the boundary lines c = 0, M carry no
// unknown and read as zero.
__device__ __forceinline__ double hat(const int* __restrict__ pos, int M, int c, int i) {
  if (c <= 0 || c >= M) return 0.0;
  const int lo = pos[c - 1], mid = pos[c], hi = pos[c + 1];
  if (i <= lo || i >= hi) return 0.0;
  return i <= mid ? double(i - lo) / double(mid - lo) : double(hi - i) / double(hi - mid);
}

// E_0(c, c + (dx, dy)) = sum over the fine nodes p in the support of hat c of
// hat_c(p) (A hat_{c+d})(p), A the interior 7-point stencil (centre 4 - kh2/2,
// E/W/N/S -1 - kh2/12, SW/NE -kh2/12); hats vanish on the boundary, which drops the
// Dirichlet neighbours.
__global__ void __launch_bounds__(256) gc_assemble_kernel(const int* __restrict__ pos, int M, double kh2,
                                                          double* __restrict__ E0c) {
  const int nc = M - 1;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)nc * nc * 9) return;
  const int c = (int)(e / 9), o = (int)(e % 9);
  const int cx = c % nc + 1, cy = c / nc + 1;
  const int qx = cx + o % 3 - 1, qy = cy + o / 3 - 1;
  double acc = 0.0;
  if (qx >= 1 && qx <= nc && qy >= 1 && qy <= nc) {
    const double cc = 4.0 - kh2 / 2.0, ce = -1.0 - kh2 / 12.0, cd = -kh2 / 12.0;
    auto hq = [&](int x, int y) { return hat(pos, M, qx, x) * hat(pos, M, qy, y); };
    for (int py = pos[cy - 1] + 1; py < pos[cy + 1]; ++py) {
      const double wy = hat(pos, M, cy, py);
      for (int px = pos[cx - 1] + 1; px < pos[cx + 1]; ++px) {
        const double wz = hat(pos, M, cx, px) * wy;
        const double aq = cc * hq(px, py) + ce * (hq(px - 1, py) + hq(px + 1, py) + hq(px, py - 1) + hq(px, py + 1)) +
                          cd * (hq(px - 1, py - 1) + hq(px + 1, py + 1));
        acc += wz * aq;
      }
    }
  }
  E0c[e] = acc;
}

// Dense level-0 blocks of block row i (coarse row i + 1): B_i (within the row),
// A_i (to row i - 1), C_i (to row i + 1), at work + (3 i + {0, 1, 2}) n^2, each stored
// transposed: entry (r, c) at c n + r.
__global__ void __launch_bounds__(256) gc_blocks_kernel(const double* __restrict__ E0c, int n,
                                                        double* __restrict__ work) {
  const long long nn = (long long)n * n;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= 3 * nn * n) return;
  const int i = (int)(e / (3 * nn));
  const long long rem = e - (long long)i * 3 * nn;
  const int which = (int)(rem / nn);
  const int c = (int)((rem % nn) / n), r = (int)(rem % n);
  const int dx = c - r, dy = which == 0 ? 0 : (which == 1 ? -1 : 1);
  double v = 0.0;
  if (dx >= -1 && dx <= 1) v = E0c[((long long)i * n + r) * 9 + 3 * (dy + 1) + (dx + 1)];
  work[e] = v;
}

// C = (acc ? C : 0) + sign * A B for every task (blockIdx.y), n x n row-major FP64,
// 64 x 64 output tile per workgroup, 4 x 4 per thread, k staged through LDS in 16s.
constexpr int kGT = 64, kGK = 16;
__global__ void __launch_bounds__(256) gc_gemm_kernel(const GemmTask* __restrict__ tasks, double* fac,
                                                      double* work, int n) {
  const GemmTask t = tasks[blockIdx.y];
  double* const base[2] = {fac, work};
  const double* __restrict__ A = base[t.arr[0]] + t.off[0];
  const double* __restrict__ B = base[t.arr[1]] + t.off[1];
  double* C = base[t.arr[2]] + t.off[2];
  const int tiles = (n + kGT - 1) / kGT;
  const int r0 = (blockIdx.x / tiles) * kGT, c0 = (blockIdx.x % tiles) * kGT;
  __shared__ double As[kGK][kGT + 1];
  __shared__ double Bs[kGK][kGT];
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < n; k0 += kGK) {
    for (int e = tid; e < kGT * kGK; e += 256) {
      const int r = e / kGK, k = e % kGK;
      As[k][r] = (r0 + r < n && k0 + k < n) ? A[(long long)(r0 + r) * n + k0 + k] : 0.0;
    }
    for (int e = tid; e < kGK * kGT; e += 256) {
      const int k = e / kGT, c = e % kGT;
      Bs[k][c] = (k0 + k < n && c0 + c < n) ? B[(long long)(k0 + k) * n + c0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kGK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty + 16 * i;
    if (r >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tx + 16 * j;
      if (c >= n) continue;
      const long long idx = (long long)r * n + c;
      C[idx] = (t.acc ? C[idx] : 0.0) + t.sign * acc[i][j];
    }
  }
}

// Largest |coefficient| of E_0 per workgroup: the scale its pivots are compared against.
constexpr int kAbsMaxBlocks = 64;
__global__ void __launch_bounds__(256) gc_absmax_kernel(const double* __restrict__ x, long long n,
                                                        double* __restrict__ out) {
  double m = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256)
    m = fmax(m, fabs(x[e]));
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, kWave));
  __shared__ double sh[256 / kWave];
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) r = fmax(r, sh[w]);
    out[blockIdx.x] = r;
  }
}

// Inverse of a work block into the factor array: copy, then Gauss-Jordan with partial
// pivoting in place (one workgroup per task).  pivmin[task] = smallest |pivot|.
constexpr int kInvThreads = 1024;
__global__ void __launch_bounds__(kInvThreads) gc_inverse_kernel(const InvTask* __restrict__ tasks,
                                                                 const double* __restrict__ work, double* fac,
                                                                 int n, double* __restrict__ pivmin) {
  const InvTask t = tasks[blockIdx.x];
  double* Am = fac + t.dst;
  const double* S = work + t.src;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  constexpr int kWaves = kInvThreads / kWave;
  __shared__ int perm[kMaxGlobalCoarse];
  __shared__ double colp[kMaxGlobalCoarse];
  __shared__ double prow[kMaxGlobalCoarse];
  __shared__ double redv[kWaves];
  __shared__ int redi[kWaves];
  for (long long e = tid; e < (long long)n * n; e += kInvThreads) Am[e] = S[e];
  __syncthreads();
  double minp = INFINITY;
  for (int p = 0; p < n; ++p) {
    double best = -1.0;
    int bi = p;
    for (int r = p + tid; r < n; r += kInvThreads) {
      const double v = fabs(Am[(long long)r * n + p]);
      if (v > best) { best = v; bi = r; }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, kWave);
      const int oi = __shfl_xor(bi, o, kWave);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { redv[wave] = best; redi[wave] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = redv[0];
      int q = redi[0];
      for (int w = 1; w < kWaves; ++w)
        if (redv[w] > b || (redv[w] == b && redi[w] < q)) { b = redv[w]; q = redi[w]; }
      perm[p] = q;
      redv[0] = b;
    }
    __syncthreads();
    const int q = perm[p];
    minp = fmin(minp, redv[0]);
    if (q != p) {
      for (int c = tid; c < n; c += kInvThreads) {
        const double x = Am[(long long)p * n + c];
        Am[(long long)p * n + c] = Am[(long long)q * n + c];
        Am[(long long)q * n + c] = x;
      }
    }
    __syncthreads();
    const double inv = 1.0 / Am[(long long)p * n + p];
    // scaled pivot row (its pivot entry becomes 1 / pivot) and the pivot column
    for (int c = tid; c < n; c += kInvThreads) {
      const double v = (c == p) ? inv : inv * Am[(long long)p * n + c];
      prow[c] = v;
    }
    for (int r = tid; r < n; r += kInvThreads) colp[r] = Am[(long long)r * n + p];
    __syncthreads();
    for (int c = tid; c < n; c += kInvThreads) Am[(long long)p * n + c] = prow[c];
    for (int r = wave; r < n; r += kWaves) {
      if (r == p) continue;
      const double f = colp[r];
      double* row = Am + (long long)r * n;
      for (int c = lane; c < n; c += kWave) row[c] = (c == p) ? -prow[p] * f : row[c] - prow[c] * f;
    }
    __syncthreads();
  }
  // undo the row interchanges by swapping columns in reverse order
  for (int p = n - 1; p >= 0; --p) {
    const int q = perm[p];
    if (q != p) {
      for (int r = tid; r < n; r += kInvThreads) {
        const double x = Am[(long long)r * n + p];
        Am[(long long)r * n + p] = Am[(long long)r * n + q];
        Am[(long long)r * n + q] = x;
      }
    }
    __syncthreads();
  }
  if (tid == 0) pivmin[blockIdx.x] = minp;
}

// One level of the block cyclic reduction solve: for task blockIdx.y and output rows
// [blockIdx.x * RPB, +RPB) of its block,
//   out = (base ? out : 0) + sum_t mat_t in_t,
// with the matrices stored transposed, so lane r of each of the 256 / RPB column slices
// reads entries (k, row0 + r) of consecutive rows: coalesced, one output row per lane,
// the slices summed through LDS at the end.  Every matrix entry is read once for all
// right-hand sides of a group of kBcrRhsGroup.  Each lane keeps CH columns of every
// term in flight per pass (chosen per launch shape by timing whole two-level solves).
template <int RPB, int NT, int CH>
__global__ void __launch_bounds__(NT) gc_bcr_kernel(const BcrTask* __restrict__ tasks, int first,
                                                    const double* __restrict__ fac, cplx<double>* cv,
                                                    long long cvstride, int n, int nrhs) {
  constexpr int S = NT / RPB;
  const BcrTask t = tasks[first + blockIdx.y];
  const int r = threadIdx.x % RPB, sl = threadIdx.x / RPB;
  const int row = blockIdx.x * RPB + r;
  const bool live = row < n;
  __shared__ double red[2][NT];
  for (int g = 0; g < nrhs; g += kBcrRhsGroup) {
    const int ng = min(kBcrRhsGroup, nrhs - g);
    double are[kBcrRhsGroup], aim[kBcrRhsGroup];
#pragma unroll
    for (int q = 0; q < kBcrRhsGroup; ++q) { are[q] = 0.0; aim[q] = 0.0; }
    if (live) {
      // tiled blocks: entry (row, k) at tile (row / kBcrTile), k kBcrTile + row % kBcrTile
      const long long roff = (long long)(row / kBcrTile) * n * kBcrTile + row % kBcrTile;
      // chunks of CH columns per lane for all terms at once, every load in flight
      // together (indices past the end are clamped and their entries zeroed, so every
      // load stays in bounds)
      for (int k0 = sl; k0 < n; k0 += CH * S) {
        double mk[3][CH];
#pragma unroll
        for (int tm = 0; tm < 3; ++tm) {
          if (tm < t.nt) {
            const double* __restrict__ m = fac + t.mat[tm] + roff;
#pragma unroll
            for (int u = 0; u < CH; ++u) mk[tm][u] = m[(long long)min(k0 + u * S, n - 1) * kBcrTile];
          }
        }
#pragma unroll
        for (int tm = 0; tm < 3; ++tm)
#pragma unroll
          for (int u = 0; u < CH; ++u)
            if (tm >= t.nt || k0 + u * S >= n) mk[tm][u] = 0.0;
#pragma unroll
        for (int q = 0; q < kBcrRhsGroup; ++q) {
          if (q < ng) {
#pragma unroll
            for (int tm = 0; tm < 3; ++tm) {
              if (tm < t.nt) {
                const cplx<double>* __restrict__ v = cv + (long long)(g + q) * cvstride + t.in[tm];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                  const cplx<double> x = v[min(k0 + u * S, n - 1)];
                  are[q] = fma(mk[tm][u], x.re, are[q]);
                  aim[q] = fma(mk[tm][u], x.im, aim[q]);
                }
              }
            }
          }
        }
      }
    }
    // sum the S column slices of each right-hand side through LDS
#pragma unroll
    for (int q = 0; q < kBcrRhsGroup; ++q) {
      if (q < ng) {
        red[0][threadIdx.x] = are[q];
        red[1][threadIdx.x] = aim[q];
        __syncthreads();
        if (sl == 0 && live) {
          double re = 0.0, im = 0.0;
          for (int j = 0; j < S; ++j) {
            re += red[0][j * RPB + r];
            im += red[1][j * RPB + r];
          }
          cplx<double>* o = cv + (long long)(g + q) * cvstride + t.out + row;
          const cplx<double> prev = t.base ? *o : czero<double>();
          *o = cplx<double>{prev.re + re, prev.im + im};
        }
        __syncthreads();
      }
    }
  }
}

// Solve layout of the factors: block b (n x n, stored transposed, b nn + k n + row) to
// kBcrTile-row tiles, b tsz + (row / kBcrTile) n kBcrTile + k kBcrTile + row % kBcrTile,
// so that a workgroup of the solve streams its rows' tile contiguously.
__global__ void __launch_bounds__(256) gc_tile_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                      int n, long long nblocks, long long tsz) {
  const long long nn = (long long)n * n;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= nblocks * nn) return;
  const long long b = e / nn;
  const int k = (int)((e % nn) / n), row = (int)(e % n);
  dst[b * tsz + (long long)(row / kBcrTile) * n * kBcrTile + (long long)k * kBcrTile + row % kBcrTile] = src[e];
}

// Level-0 couplings applied directly from the coarse operator's rows:
//   out -= A_row in0 + C_row in1,
// A_row / C_row the tridiagonal couplings of block row `row` to the rows below / above
// (E_0 coefficients with dy = -1 / +1).  One thread per entry, grid z over right-hand sides.
__global__ void __launch_bounds__(256) gc_sparse_kernel(const SpTask* __restrict__ tasks, int first,
                                                        const double* __restrict__ E0c, cplx<double>* cv,
                                                        long long cvstride, int n) {
  const SpTask t = tasks[first + blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  cplx<double>* base = cv + (long long)blockIdx.z * cvstride;
  cplx<double> acc = base[t.out + j];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    if (!t.has[side]) continue;
    const double* cf = E0c + ((long long)t.row * n + j) * 9 + (side ? 6 : 0);
    const cplx<double>* v = base + t.in[side];
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int jj = j + dx;
      if (jj < 0 || jj >= n) continue;
      acc = acc - cf[dx + 1] * v[jj];
    }
  }
  base[t.out + j] = acc;
}

// b = Z_0^T r: one thread per coarse unknown, summing its hat's support.
__global__ void __launch_bounds__(256) gc_restrict_kernel(const int* __restrict__ pos, int M, int N,
                                                          const cplx<double>* __restrict__ r, long long rstride,
                                                          const int* jdev, long long rslot,
                                                          const int* __restrict__ done, cplx<double>* __restrict__ cv,
                                                          long long cvstride) {
  const int rhs = blockIdx.y;
  if (done && done[rhs]) return;
  const int nc = M - 1;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc * nc) return;
  const int cx = c % nc + 1, cy = c / nc + 1;
  const long long js = jdev ? (long long)*jdev : 0;
  const cplx<double>* __restrict__ x = r + js * rslot + (long long)rhs * rstride;
  const int ld = N - 1;
  cplx<double> acc = czero<double>();
  for (int py = pos[cy - 1] + 1; py < pos[cy + 1]; ++py) {
    const double wy = hat(pos, M, cy, py);
    for (int px = pos[cx - 1] + 1; px < pos[cx + 1]; ++px) {
      const double wz = wy * hat(pos, M, cx, px);
      const cplx<double> v = x[(long long)(py - 1) * ld + (px - 1)];
      acc.re = fma(wz, v.re, acc.re);
      acc.im = fma(wz, v.im, acc.im);
    }
  }
  cv[(long long)rhs * cvstride + c] = acc;
}

// q = Z_0 x at every fine node: bilinear in the coarse cell (cell[i], cell[j]).
__global__ void __launch_bounds__(256) gc_prolong_kernel(const int* __restrict__ pos, const int* __restrict__ cell,
                                                         int M, int N, const cplx<double>* __restrict__ cv,
                                                         long long cvstride, long long xoff,
                                                         const int* __restrict__ done, cplx<double>* __restrict__ q,
                                                         long long qstride) {
  const int rhs = blockIdx.z;
  if (done && done[rhs]) return;
  const int m = N - 1, nc = M - 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y * blockDim.y + threadIdx.y + 1;
  if (i > m || j > m) return;
  const cplx<double>* __restrict__ X = cv + (long long)rhs * cvstride + xoff;
  const int ci = cell[i], cj = cell[j];
  const double tx = double(i - pos[ci]) / double(pos[ci + 1] - pos[ci]);
  const double ty = double(j - pos[cj]) / double(pos[cj + 1] - pos[cj]);
  const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty};
  cplx<double> acc = czero<double>();
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int cyy = cj + b;
    if (cyy < 1 || cyy > nc) continue;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int cxx = ci + a;
      if (cxx < 1 || cxx > nc) continue;
      const cplx<double> v = X[(long long)(cyy - 1) * nc + (cxx - 1)];
      acc = acc + (wx[a] * wy[b]) * v;
    }
  }
  q[(long long)rhs * qstride + (long long)(j - 1) * m + (i - 1)] = acc;
}

// w = r - A q (global interior stencil).
__global__ void __launch_bounds__(256) gc_residual_kernel(double kh2, int N, const cplx<double>* __restrict__ r,
                                                          long long rstride, const int* jdev, long long rslot,
                                                          const cplx<double>* __restrict__ q, long long qstride,
                                                          const int* __restrict__ done, cplx<double>* __restrict__ w,
                                                          long long wstride) {
  const int rhs = blockIdx.z;
  if (done && done[rhs]) return;
  const int m = N - 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= m || j >= m) return;
  const double cc = 4.0 - kh2 / 2.0, ce = -1.0 - kh2 / 12.0, cd = -kh2 / 12.0;
  const cplx<double>* __restrict__ x = q + (long long)rhs * qstride;
  const long long nidx = (long long)j * m + i;
  cplx<double> side = czero<double>(), diag = czero<double>();
  if (i > 0) side = side + x[nidx - 1];
  if (i < m - 1) side = side + x[nidx + 1];
  if (j > 0) side = side + x[nidx - m];
  if (j < m - 1) side = side + x[nidx + m];
  if (i > 0 && j > 0) diag = diag + x[nidx - m - 1];
  if (i < m - 1 && j < m - 1) diag = diag + x[nidx + m + 1];
  const cplx<double> aq = cc * x[nidx] + ce * side + cd * diag;
  const long long js = jdev ? (long long)*jdev : 0;
  const cplx<double> rv = r[js * rslot + (long long)rhs * rstride + nidx];
  w[(long long)rhs * wstride + nidx] = rv - aq;
}

struct LevelPlan {
  std::vector<InvTask> inv;
  std::vector<GemmTask> g1, g2, g3;
};

}  // namespace

template <typename T>
hipError_t GlobalCoarse::alloc(T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  allocs.push_back(q);
  *p = (T*)q;
  return hipSuccess;
}

GlobalCoarse::~GlobalCoarse() {
  for (void* p : allocs) (void)hipFree(p);
}

#define GC_TRY(x)                        \
  do {                                   \
    hipError_t e_ = (x);                 \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

hipError_t GlobalCoarse::setup(int n, int m, double k, int nr, hipStream_t st) {
  n_fine = n;
  M = m;
  nc = m - 1;
  ncoarse = (long long)nc * nc;
  ndof = (long long)(n - 1) * (n - 1);
  nrhs = nr;
  const double h = 1.0 / n;
  kh2 = (k * h) * (k * h);
  const int nb = nc, bn = nc;
  const long long nn = (long long)bn * bn;
  // coarse grid lines and the coarse interval of each fine index
  std::vector<int> pos_h(m + 1), cell_h(n + 1);
  for (int c = 0; c <= m; ++c) pos_h[c] = (int)((2LL * c * n + m) / (2LL * m));
  for (int c = 0; c < m; ++c)
    for (int i = pos_h[c]; i < pos_h[c + 1]; ++i) cell_h[i] = c;
  cell_h[n] = m - 1;
  GC_TRY(alloc(&pos, m + 1));
  GC_TRY(alloc(&cell, n + 1));
  GC_TRY(hipMemcpyAsync(pos, pos_h.data(), sizeof(int) * (m + 1), hipMemcpyHostToDevice, st));
  GC_TRY(hipMemcpyAsync(cell, cell_h.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st));
  GC_TRY(alloc(&E0c, (size_t)ncoarse * 9));
  {
    const long long tot = ncoarse * 9;
    hipLaunchKernelGGL(gc_assemble_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, pos, m, kh2, E0c);
    GC_TRY(hipGetLastError());
    GC_TRY(alloc(&emax_d, kAbsMaxBlocks));
    hipLaunchKernelGGL(gc_absmax_kernel, dim3(kAbsMaxBlocks), dim3(256), 0, st, (const double*)E0c, tot, emax_d);
    GC_TRY(hipGetLastError());
  }
  GC_TRY(alloc(&cv, (size_t)nr * 2 * ncoarse));
  GC_TRY(alloc(&q, (size_t)nr * ndof));
  GC_TRY(alloc(&w, (size_t)nr * ndof));

  // ---- plan the block cyclic reduction ----
  // Work blocks: B_i, A_i, C_i per block row, then the level-0 products Fm_i, Fp_i that
  // only the set-up needs.
  auto Bw = [&](int i) { return 3LL * i * nn; };
  auto Aw = [&](int i) { return (3LL * i + 1) * nn; };
  auto Cw = [&](int i) { return (3LL * i + 2) * nn; };
  auto bvec = [&](int i) { return i * bn; };
  auto xvec = [&](int i) { return (int)(ncoarse + (long long)i * bn); };
  long long nf = 0, nw = 3LL * nb * nn;
  auto newfac = [&]() { const long long o = nf; nf += nn; return o; };
  auto newwork = [&]() { const long long o = nw; nw += nn; return o; };
  // Every block is stored transposed (column-major), which lets the solve kernel give
  // each lane an output row with coalesced loads and no cross-lane reduction; a product
  // X Y of true blocks is then the stored product Y^T X^T.
  auto mul = [](std::vector<GemmTask>& v, long long x, int xa, long long y, int ya, long long c, int ca, int acc,
                double sign) { v.push_back(GemmTask{{y, x, c}, {ya, xa, ca}, acc, sign}); };
  std::vector<LevelPlan> plans;
  // solve launches: dense (BcrTask) or sparse (SpTask) phases, reductions upward
  std::vector<std::pair<int, std::vector<BcrTask>>> red_dense, back_dense;   // (level, tasks)
  std::vector<SpTask> red0_sparse, back0_sparse;
  std::vector<BcrTask> red0_dense, back0_dense, top;
  std::vector<int> act(nb);
  for (int i = 0; i < nb; ++i) act[i] = i;
  std::vector<char> hasA(nb), hasC(nb);
  for (int i = 0; i < nb; ++i) { hasA[i] = i > 0; hasC[i] = i < nb - 1; }
  std::vector<long long> binv(nb, -1);
  for (int level = 0;; ++level) {
    const int cnt = (int)act.size();
    LevelPlan lp;
    if (cnt == 1) {
      const int rt = act[0];
      binv[rt] = newfac();
      lp.inv.push_back(InvTask{Bw(rt), binv[rt]});
      plans.push_back(lp);
      BcrTask tk{};
      tk.nt = 1; tk.mat[0] = binv[rt]; tk.in[0] = bvec(rt); tk.out = xvec(rt); tk.base = 0;
      top.push_back(tk);
      break;
    }
    // On level 0 the couplings A_i, C_i are the coarse operator's tridiagonal rows, so the
    // solve applies them directly (sparse phases) and keeps only Binv_e: the reduction
    // forms y_e = Binv_e b_e (into x_e, as scratch) and b_i -= A_i y_{i-1} + C_i y_{i+1};
    // the back substitution forms b_e -= A_e x_{e-1} + C_e x_{e+1} and x_e = Binv_e b_e.
    const bool sparse = level == 0;
    std::vector<BcrTask> rl, bl;
    for (int p = 1; p < cnt; p += 2) {
      const int e = act[p];
      binv[e] = newfac();
      lp.inv.push_back(InvTask{Bw(e), binv[e]});
      BcrTask tk{};
      tk.out = xvec(e); tk.base = 0;
      tk.mat[0] = binv[e]; tk.in[0] = bvec(e); tk.nt = 1;
      if (sparse) {
        red0_dense.push_back(tk);
        back0_dense.push_back(tk);
        SpTask sk{};
        sk.out = bvec(e); sk.row = e;
        sk.in[0] = xvec(act[p - 1]); sk.has[0] = 1;
        if (p + 1 < cnt) { sk.in[1] = xvec(act[p + 1]); sk.has[1] = 1; }
        back0_sparse.push_back(sk);
        continue;
      }
      const long long P = newfac();
      mul(lp.g1, binv[e], 0, Aw(e), 1, P, 0, 0, -1.0);
      tk.mat[tk.nt] = P; tk.in[tk.nt] = xvec(act[p - 1]); tk.nt++;
      if (p + 1 < cnt) {
        const long long R = newfac();
        mul(lp.g1, binv[e], 0, Cw(e), 1, R, 0, 0, -1.0);
        tk.mat[tk.nt] = R; tk.in[tk.nt] = xvec(act[p + 1]); tk.nt++;
      }
      bl.push_back(tk);
    }
    std::vector<int> kept;
    std::vector<char> nA, nC;
    const int fa = sparse ? 1 : 0;   // Fm, Fp: set-up work blocks on level 0, factors above
    for (int p = 0; p < cnt; p += 2) {
      const int i = act[p];
      BcrTask tk{};
      tk.out = bvec(i); tk.base = 1; tk.nt = 0;
      SpTask sk{};
      sk.out = bvec(i); sk.row = i;
      bool newA = false, newC = false;
      if (p >= 1) {
        const int em = act[p - 1];
        const long long Fm = sparse ? newwork() : newfac();
        mul(lp.g1, Aw(i), 1, binv[em], 0, Fm, fa, 0, -1.0);
        mul(lp.g2, Fm, fa, Cw(em), 1, Bw(i), 1, 1, 1.0);
        if (hasA[em]) {
          mul(lp.g2, Fm, fa, Aw(em), 1, Aw(i), 1, 0, 1.0);
          newA = true;
        }
        tk.mat[tk.nt] = Fm; tk.in[tk.nt] = bvec(em); tk.nt++;
        sk.in[0] = xvec(em); sk.has[0] = 1;
      }
      if (p + 1 < cnt) {
        const int ep = act[p + 1];
        const long long Fp = sparse ? newwork() : newfac();
        mul(lp.g1, Cw(i), 1, binv[ep], 0, Fp, fa, 0, -1.0);
        mul(lp.g3, Fp, fa, Aw(ep), 1, Bw(i), 1, 1, 1.0);
        if (hasC[ep]) {
          mul(lp.g2, Fp, fa, Cw(ep), 1, Cw(i), 1, 0, 1.0);
          newC = true;
        }
        tk.mat[tk.nt] = Fp; tk.in[tk.nt] = bvec(ep); tk.nt++;
        sk.in[1] = xvec(ep); sk.has[1] = 1;
      }
      if (sparse) {
        if (sk.has[0] || sk.has[1]) red0_sparse.push_back(sk);
      } else if (tk.nt) {
        rl.push_back(tk);
      }
      kept.push_back(i);
      nA.push_back(newA);
      nC.push_back(newC);
    }
    for (size_t t = 0; t < kept.size(); ++t) { hasA[kept[t]] = nA[t]; hasC[kept[t]] = nC[t]; }
    plans.push_back(lp);
    if (!sparse) {
      red_dense.emplace_back(level, rl);
      back_dense.emplace_back(level, bl);
    }
    act = kept;
  }
  nfac = nf;
  // solve phases in order: level-0 reduction (dense, sparse), higher reductions, the top,
  // higher back substitutions downward, level-0 back substitution (sparse, dense)
  std::vector<BcrTask> all;
  std::vector<SpTask> all_sp;
  phases.clear();
  auto add_dense = [&](const std::vector<BcrTask>& v) {
    if (v.empty()) return;
    phases.push_back(BcrPhase{(int)all.size(), (int)v.size(), 0});
    all.insert(all.end(), v.begin(), v.end());
  };
  auto add_sparse = [&](const std::vector<SpTask>& v) {
    if (v.empty()) return;
    phases.push_back(BcrPhase{(int)all_sp.size(), (int)v.size(), 1});
    all_sp.insert(all_sp.end(), v.begin(), v.end());
  };
  add_dense(red0_dense);
  add_sparse(red0_sparse);
  for (auto& v : red_dense) add_dense(v.second);
  add_dense(top);
  for (int l = (int)back_dense.size() - 1; l >= 0; --l) add_dense(back_dense[l].second);
  add_sparse(back0_sparse);
  add_dense(back0_dense);
  solve_bytes_ = 0;
  for (const BcrTask& tk : all) solve_bytes_ += (long long)tk.nt * nn * 8 + (long long)(tk.nt + 1 + tk.base) * bn * 16;
  for (const SpTask& sk : all_sp)
    solve_bytes_ += (long long)(sk.has[0] + sk.has[1]) * bn * (3 * 8 + 16) + 2LL * bn * 16;

  // ---- factor on the device ----
  // The set-up works on plain n x n blocks (sfac); the solve reads them re-laid in row
  // tiles (fac): block b moves from offset b nn to b tsz.
  const long long nblk = nfac / nn, tsz = (long long)((bn + kBcrTile - 1) / kBcrTile) * kBcrTile * bn;
  for (BcrTask& tk : all)
    for (int q = 0; q < tk.nt; ++q) tk.mat[q] = (tk.mat[q] / nn) * tsz;
  GC_TRY(alloc(&fac, (size_t)(nblk * tsz)));
  GC_TRY(alloc(&tasks, all.size()));
  GC_TRY(hipMemcpyAsync(tasks, all.data(), sizeof(BcrTask) * all.size(), hipMemcpyHostToDevice, st));
  GC_TRY(alloc(&sptasks, std::max<size_t>(all_sp.size(), 1)));
  if (!all_sp.empty())
    GC_TRY(hipMemcpyAsync(sptasks, all_sp.data(), sizeof(SpTask) * all_sp.size(), hipMemcpyHostToDevice, st));
  size_t ninv = 0, ngemm = 0, maxg = 0, maxi = 0;
  for (auto& lp : plans) {
    ninv += lp.inv.size();
    maxi = std::max(maxi, lp.inv.size());
    ngemm += lp.g1.size() + lp.g2.size() + lp.g3.size();
    maxg = std::max({maxg, lp.g1.size(), lp.g2.size(), lp.g3.size()});
  }
  double* work = nullptr;
  InvTask* dinv = nullptr;
  GemmTask* dgemm = nullptr;
  double* dpiv = nullptr;
  double* sfac = nullptr;
  hipError_t err = hipMalloc(&work, sizeof(double) * (size_t)nw);
  if (err == hipSuccess) err = hipMalloc(&sfac, sizeof(double) * (size_t)nfac);
  if (err == hipSuccess) err = hipMalloc(&dinv, sizeof(InvTask) * std::max<size_t>(ninv, 1));
  if (err == hipSuccess) err = hipMalloc(&dgemm, sizeof(GemmTask) * std::max<size_t>(ngemm, 1));
  if (err == hipSuccess) err = hipMalloc(&dpiv, sizeof(double) * std::max<size_t>(ninv, 1));
  std::vector<InvTask> inv_all;
  std::vector<GemmTask> gemm_all;
  for (auto& lp : plans) {
    inv_all.insert(inv_all.end(), lp.inv.begin(), lp.inv.end());
    gemm_all.insert(gemm_all.end(), lp.g1.begin(), lp.g1.end());
    gemm_all.insert(gemm_all.end(), lp.g2.begin(), lp.g2.end());
    gemm_all.insert(gemm_all.end(), lp.g3.begin(), lp.g3.end());
  }
  if (err == hipSuccess)
    err = hipMemcpyAsync(dinv, inv_all.data(), sizeof(InvTask) * inv_all.size(), hipMemcpyHostToDevice, st);
  if (err == hipSuccess && !gemm_all.empty())
    err = hipMemcpyAsync(dgemm, gemm_all.data(), sizeof(GemmTask) * gemm_all.size(), hipMemcpyHostToDevice, st);
  if (err == hipSuccess) {
    const long long tot = 3LL * nb * nn;
    hipLaunchKernelGGL(gc_blocks_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, (const double*)E0c,
                       bn, work);
    err = hipGetLastError();
  }
  const int tiles = (bn + kGT - 1) / kGT;
  size_t io = 0, go = 0;
  for (auto& lp : plans) {
    if (err != hipSuccess) break;
    hipLaunchKernelGGL(gc_inverse_kernel, dim3((unsigned)lp.inv.size()), dim3(kInvThreads), 0, st, dinv + io,
                       (const double*)work, sfac, bn, dpiv + io);
    err = hipGetLastError();
    io += lp.inv.size();
    for (const auto* g : {&lp.g1, &lp.g2, &lp.g3}) {
      if (err != hipSuccess || g->empty()) continue;
      hipLaunchKernelGGL(gc_gemm_kernel, dim3((unsigned)(tiles * tiles), (unsigned)g->size()), dim3(256), 0, st,
                         dgemm + go, sfac, work, bn);
      err = hipGetLastError();
      go += g->size();
    }
  }
  if (err == hipSuccess) {
    const long long tot = nblk * nn;
    hipLaunchKernelGGL(gc_tile_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, (const double*)sfac, fac,
                       bn, nblk, tsz);
    err = hipGetLastError();
  }
  std::vector<double> piv(ninv, 0.0), emax(kAbsMaxBlocks, 0.0);
  if (err == hipSuccess) err = hipMemcpyAsync(piv.data(), dpiv, sizeof(double) * ninv, hipMemcpyDeviceToHost, st);
  if (err == hipSuccess)
    err = hipMemcpyAsync(emax.data(), emax_d, sizeof(double) * kAbsMaxBlocks, hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  (void)hipFree(sfac);
  (void)hipFree(work);
  (void)hipFree(dinv);
  (void)hipFree(dgemm);
  (void)hipFree(dpiv);
  if (err != hipSuccess) return err;
  // smallest |pivot| over every block inverse; a non-finite one marks the factor unusable
  bool finite = !piv.empty();
  min_pivot = INFINITY;
  for (double v : piv) {
    finite = finite && std::isfinite(v);
    min_pivot = std::min(min_pivot, v);
  }
  if (!finite) min_pivot = 0.0;
  max_entry = *std::max_element(emax.begin(), emax.end());
  return hipSuccess;
}

hipError_t GlobalCoarse::restrict_rhs(const cplx<double>* r, long long rstride, const int* jdev, long long rslot,
                                      const int* done, int nr, hipStream_t st) {
  dim3 grd((unsigned)((ncoarse + 255) / 256), (unsigned)nr);
  hipLaunchKernelGGL(gc_restrict_kernel, grd, dim3(256), 0, st, (const int*)pos, M, n_fine, r, rstride, jdev, rslot,
                     done, cv, 2 * ncoarse);
  return hipGetLastError();
}

hipError_t GlobalCoarse::solve(int nr, hipStream_t st) {
  for (const BcrPhase& ph : phases) {
    if (ph.kind == 1) {
      hipLaunchKernelGGL(gc_sparse_kernel, dim3((unsigned)((nc + 255) / 256), (unsigned)ph.count, (unsigned)nr),
                         dim3(256), 0, st, (const SpTask*)sptasks, ph.first, (const double*)E0c, cv, 2 * ncoarse, nc);
      GC_TRY(hipGetLastError());
      continue;
    }
    // Rows per workgroup and columns in flight per lane (measured on the k = 200, N = 637,
    // M = 318 solve): 64 rows (4 column slices, 16 columns each) when the level has many
    // tasks, 16 (16 slices, 5 columns) down to 8 tasks, 4 (64 slices, 5 columns) on the last
    // levels, where the launch is bound by load latency.  A pass then covers 64, 80 and 320
    // columns: whole passes over the 317 columns of that solve, and 2.6x the loads in flight
    // of 8 columns per lane at the widest shape (coarse solve 0.49 -> 0.34 ms).
    const long long c = ph.count;
    if (c * ((nc + 63) / 64) >= 384) {
      hipLaunchKernelGGL((gc_bcr_kernel<64, 256, 16>), dim3((unsigned)((nc + 63) / 64), (unsigned)c), dim3(256), 0, st,
                         (const BcrTask*)tasks, ph.first, (const double*)fac, cv, 2 * ncoarse, nc, nr);
    } else if (c >= 8) {
      hipLaunchKernelGGL((gc_bcr_kernel<16, 256, 5>), dim3((unsigned)((nc + 15) / 16), (unsigned)c), dim3(256), 0, st,
                         (const BcrTask*)tasks, ph.first, (const double*)fac, cv, 2 * ncoarse, nc, nr);
    } else {
      hipLaunchKernelGGL((gc_bcr_kernel<4, 256, 5>), dim3((unsigned)((nc + 3) / 4), (unsigned)c), dim3(256), 0, st,
                         (const BcrTask*)tasks, ph.first, (const double*)fac, cv, 2 * ncoarse, nc, nr);
    }
    GC_TRY(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t GlobalCoarse::correct(const cplx<double>* r, long long rstride, const int* jdev, long long rslot,
                                 const int* done, int nr, hipStream_t st) {
  const int mm = n_fine - 1;
  dim3 blk(64, 4);
  dim3 grd((mm + 63) / 64, (mm + 3) / 4, nr);
  hipLaunchKernelGGL(gc_prolong_kernel, grd, blk, 0, st, (const int*)pos, (const int*)cell, M, n_fine,
                     (const cplx<double>*)cv, 2 * ncoarse, ncoarse, done, q, ndof);
  GC_TRY(hipGetLastError());
  hipLaunchKernelGGL(gc_residual_kernel, grd, blk, 0, st, kh2, n_fine, r, rstride, jdev, rslot,
                     (const cplx<double>*)q, ndof, done, w, ndof);
  return hipGetLastError();
}

}  // namespace ddh
