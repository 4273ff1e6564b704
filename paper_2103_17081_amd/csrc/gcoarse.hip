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
// A_i (to row i - 1), C_i (to row i + 1), at work + (3 i + {0, 1, 2}) n^2.
__global__ void __launch_bounds__(256) gc_blocks_kernel(const double* __restrict__ E0c, int n,
                                                        double* __restrict__ work) {
  const long long nn = (long long)n * n;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= 3 * nn * n) return;
  const int i = (int)(e / (3 * nn));
  const long long rem = e - (long long)i * 3 * nn;
  const int which = (int)(rem / nn);
  const int r = (int)((rem % nn) / n), c = (int)(rem % n);
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

// Inverse of a work block into the factor array: copy, then Gauss-Jordan with partial
// pivoting in place (one workgroup per task).  pivmin[task] = smallest |pivot|.
constexpr int kInvThreads = 512;
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

// One level of the block cyclic reduction solve: for task blockIdx.y and rows
// [blockIdx.x * 4 rpw, +4 rpw) of its output block,
//   out = (base ? out : 0) + sum_t mat_t in_t,
// one wave per row (lanes stride over the columns), all right-hand sides per matrix
// read, in groups of kBcrRhsGroup.
__global__ void __launch_bounds__(256) gc_bcr_kernel(const BcrTask* __restrict__ tasks, int first,
                                                     const double* __restrict__ fac, cplx<double>* cv,
                                                     long long cvstride, int n, int nrhs, int rpw) {
  const BcrTask t = tasks[first + blockIdx.y];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int rbase = (blockIdx.x * 4 + wave) * rpw;
  for (int rr = 0; rr < rpw; ++rr) {
    const int row = rbase + rr;
    if (row >= n) break;
    for (int g = 0; g < nrhs; g += kBcrRhsGroup) {
      const int ng = min(kBcrRhsGroup, nrhs - g);
      double are[kBcrRhsGroup], aim[kBcrRhsGroup];
#pragma unroll
      for (int s = 0; s < kBcrRhsGroup; ++s) { are[s] = 0.0; aim[s] = 0.0; }
      for (int term = 0; term < t.nt; ++term) {
        const double* __restrict__ m = fac + t.mat[term] + (long long)row * n;
        const cplx<double>* __restrict__ v = cv + (long long)g * cvstride + t.in[term];
        for (int c = lane; c < n; c += kWave) {
          const double a = m[c];
#pragma unroll
          for (int s = 0; s < kBcrRhsGroup; ++s) {
            if (s < ng) {
              const cplx<double> x = v[(long long)s * cvstride + c];
              are[s] = fma(a, x.re, are[s]);
              aim[s] = fma(a, x.im, aim[s]);
            }
          }
        }
      }
#pragma unroll
      for (int s = 0; s < kBcrRhsGroup; ++s) {
        if (s < ng) {
          const double re = wave_sum(are[s]), im = wave_sum(aim[s]);
          if (lane == 0) {
            cplx<double>* o = cv + (long long)(g + s) * cvstride + t.out + row;
            const cplx<double> prev = t.base ? *o : czero<double>();
            *o = cplx<double>{prev.re + re, prev.im + im};
          }
        }
      }
    }
  }
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
  }
  GC_TRY(alloc(&cv, (size_t)nr * 2 * ncoarse));
  GC_TRY(alloc(&q, (size_t)nr * ndof));
  GC_TRY(alloc(&w, (size_t)nr * ndof));

  // ---- plan the block cyclic reduction ----
  auto Bw = [&](int i) { return 3LL * i * nn; };
  auto Aw = [&](int i) { return (3LL * i + 1) * nn; };
  auto Cw = [&](int i) { return (3LL * i + 2) * nn; };
  auto bvec = [&](int i) { return i * bn; };
  auto xvec = [&](int i) { return (int)(ncoarse + (long long)i * bn); };
  long long nf = 0;
  auto newfac = [&]() { const long long o = nf; nf += nn; return o; };
  std::vector<LevelPlan> plans;
  std::vector<std::vector<BcrTask>> red, back;
  std::vector<BcrTask> top;
  std::vector<int> act(nb);
  for (int i = 0; i < nb; ++i) act[i] = i;
  std::vector<char> hasA(nb), hasC(nb);
  for (int i = 0; i < nb; ++i) { hasA[i] = i > 0; hasC[i] = i < nb - 1; }
  std::vector<long long> binv(nb, -1);
  while (true) {
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
    std::vector<BcrTask> rl, bl;
    for (int p = 1; p < cnt; p += 2) {
      const int e = act[p];
      binv[e] = newfac();
      lp.inv.push_back(InvTask{Bw(e), binv[e]});
      BcrTask tk{};
      tk.out = xvec(e); tk.base = 0;
      tk.mat[0] = binv[e]; tk.in[0] = bvec(e); tk.nt = 1;
      const long long P = newfac();
      lp.g1.push_back(GemmTask{{binv[e], Aw(e), P}, {0, 1, 0}, 0, -1.0});
      tk.mat[tk.nt] = P; tk.in[tk.nt] = xvec(act[p - 1]); tk.nt++;
      if (p + 1 < cnt) {
        const long long R = newfac();
        lp.g1.push_back(GemmTask{{binv[e], Cw(e), R}, {0, 1, 0}, 0, -1.0});
        tk.mat[tk.nt] = R; tk.in[tk.nt] = xvec(act[p + 1]); tk.nt++;
      }
      bl.push_back(tk);
    }
    std::vector<int> kept;
    std::vector<char> nA, nC;
    for (int p = 0; p < cnt; p += 2) {
      const int i = act[p];
      BcrTask tk{};
      tk.out = bvec(i); tk.base = 1; tk.nt = 0;
      bool newA = false, newC = false;
      if (p >= 1) {
        const int em = act[p - 1];
        const long long Fm = newfac();
        lp.g1.push_back(GemmTask{{Aw(i), binv[em], Fm}, {1, 0, 0}, 0, -1.0});
        lp.g2.push_back(GemmTask{{Fm, Cw(em), Bw(i)}, {0, 1, 1}, 1, 1.0});
        if (hasA[em]) {
          lp.g2.push_back(GemmTask{{Fm, Aw(em), Aw(i)}, {0, 1, 1}, 0, 1.0});
          newA = true;
        }
        tk.mat[tk.nt] = Fm; tk.in[tk.nt] = bvec(em); tk.nt++;
      }
      if (p + 1 < cnt) {
        const int ep = act[p + 1];
        const long long Fp = newfac();
        lp.g1.push_back(GemmTask{{Cw(i), binv[ep], Fp}, {1, 0, 0}, 0, -1.0});
        lp.g3.push_back(GemmTask{{Fp, Aw(ep), Bw(i)}, {0, 1, 1}, 1, 1.0});
        if (hasC[ep]) {
          lp.g2.push_back(GemmTask{{Fp, Cw(ep), Cw(i)}, {0, 1, 1}, 0, 1.0});
          newC = true;
        }
        tk.mat[tk.nt] = Fp; tk.in[tk.nt] = bvec(ep); tk.nt++;
      }
      if (tk.nt) rl.push_back(tk);
      kept.push_back(i);
      nA.push_back(newA);
      nC.push_back(newC);
    }
    for (size_t t = 0; t < kept.size(); ++t) { hasA[kept[t]] = nA[t]; hasC[kept[t]] = nC[t]; }
    plans.push_back(lp);
    red.push_back(rl);
    back.push_back(bl);
    act = kept;
  }
  nfac = nf;
  // solve phases: reductions upward, the top, back substitutions downward
  std::vector<BcrTask> all;
  phases.clear();
  auto add_phase = [&](const std::vector<BcrTask>& v) {
    if (v.empty()) return;
    phases.push_back(BcrPhase{(int)all.size(), (int)v.size()});
    all.insert(all.end(), v.begin(), v.end());
  };
  for (auto& v : red) add_phase(v);
  add_phase(top);
  for (int l = (int)back.size() - 1; l >= 0; --l) add_phase(back[l]);
  solve_bytes_ = 0;
  for (const BcrTask& tk : all) solve_bytes_ += (long long)tk.nt * nn * 8 + (long long)(tk.nt + 1 + tk.base) * bn * 16;

  // ---- factor on the device ----
  GC_TRY(alloc(&fac, (size_t)nfac));
  GC_TRY(alloc(&tasks, all.size()));
  GC_TRY(hipMemcpyAsync(tasks, all.data(), sizeof(BcrTask) * all.size(), hipMemcpyHostToDevice, st));
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
  hipError_t err = hipMalloc(&work, sizeof(double) * (size_t)(3 * nb) * nn);
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
                       (const double*)work, fac, bn, dpiv + io);
    err = hipGetLastError();
    io += lp.inv.size();
    for (const auto* g : {&lp.g1, &lp.g2, &lp.g3}) {
      if (err != hipSuccess || g->empty()) continue;
      hipLaunchKernelGGL(gc_gemm_kernel, dim3((unsigned)(tiles * tiles), (unsigned)g->size()), dim3(256), 0, st,
                         dgemm + go, fac, work, bn);
      err = hipGetLastError();
      go += g->size();
    }
  }
  std::vector<double> piv(ninv, 0.0);
  if (err == hipSuccess) err = hipMemcpyAsync(piv.data(), dpiv, sizeof(double) * ninv, hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
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
    // rows per wave: spread small levels over more workgroups
    int rpw = 4;
    while (rpw > 1 && (long long)ph.count * ((nc + 4 * rpw - 1) / (4 * rpw)) < 1024) rpw /= 2;
    const unsigned gx = (unsigned)((nc + 4 * rpw - 1) / (4 * rpw));
    hipLaunchKernelGGL(gc_bcr_kernel, dim3(gx, (unsigned)ph.count), dim3(256), 0, st, (const BcrTask*)tasks,
                       ph.first, (const double*)fac, cv, 2 * ncoarse, nc, nr, rpw);
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
