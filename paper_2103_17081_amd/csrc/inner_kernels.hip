// Batched inexact subdomain solves: GMRES on the deflated systems P_j B_j x = P_j f_j
// (Sec. 2, eq. 4; Sec. 3), all subdomains and right-hand sides in one launch.
//
// One workgroup carries one (subdomain, right-hand side) pair through its whole
// solve -- gather, deflated-operator applications, delayed-CGS2 Arnoldi with Givens
// rotations, its own convergence test, solution recovery, scatter -- so solves of
// uneven size and uneven iteration count run side by side without host round trips.
// Fine-level vectors are in the template precision T; the coarse solve is FP64.
//
// Per solve, with f = R_j r:
//   P f = f - B Z E^{-1} Z^T f,   reference norm ||P f||;
//   optional guess g accepted iff ||P f - P B g|| < ||P f||, else x0 = 0;
//   Arnoldi on the deflated operator P B with classical Gram-Schmidt applied twice in
//   the delayed form of Swirydowicz, Langou, Ananthan, Yang and Thomas (2020): the
//   operator is applied to the candidate u~_j before its second orthogonalisation, and
//   u~_j = V_j s + alpha_j v_j, so P B U~_k = V_{k+1} H_k with U~_k = V_k T_k (T upper
//   triangular, column j = (s, alpha_j));
//   stop when the least-squares residual estimate <= tol * ||P f||;
//   x = x0 + U~ y = x0 + V (T y),  u = x + Z E^{-1} Z^T (f - B x)   (so f - B u = P (f - B x));
//   the coarse vector of the recovery is assembled from those the solve already formed,
//   E^{-1} Z^T (f - B x) = E^{-1} Z^T f - E^{-1} Z^T B x0 - sum_i y_i E^{-1} Z^T B u~_i,
//   so it costs no deflated application of its own;
//   z(owned nodes of j) = u.
#include <algorithm>

#include "coarse.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace ddh {

namespace {

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

template <typename T>
struct Lds {
  cplx<T>* A;          // fine tile (stencil input)
  cplx<T>* B;          // fine tile (stencil output / working vector)
  cplx<T>* tab;        // 9 row classes x 7 coefficients
  cplx<T>* red;        // wave partial sums, (threads / wave) x stride
  cplx<T>* hT;         // update coefficients of the new basis vector (s / alpha); then T y
  cplx<T>* hU;         // update coefficients of the next candidate
  cplx<double>* sv;    // V_j^H u~_j, then |u~_j|^2
  cplx<double>* cv;    // V_j^H w, u~_j^H w, |w|^2
  cplx<double>* ct;    // coarse right-hand side
  cplx<double>* ca;    // coarse solution
  cplx<double>* lc;    // lower couplings of E staged for the coarse solve (3 per coarse node)
  cplx<double>* h;     // Hessenberg column (maxit + 2)
  cplx<double>* g;     // rotated right-hand side (maxit + 1)
  cplx<double>* sn;    // Givens sines (maxit)
  double* cs;          // Givens cosines (maxit)
  double* scal;        // 8 scalars
  int* ctrl;           // 4 ints
  int stride;          // maxit + 2
};

template <typename T>
__host__ __device__ size_t lds_bytes(int max_nj, int max_nc, int maxit, int nt) {
  const size_t s = (size_t)maxit + 2;
  size_t b = 0;
  b += 2 * align16((size_t)max_nj * sizeof(cplx<T>));
  b += align16(kClasses * kStencilPts * sizeof(cplx<T>));
  b += align16((size_t)(nt / kWave) * s * sizeof(cplx<T>));
  b += 2 * align16(s * sizeof(cplx<T>));
  b += 2 * align16(s * sizeof(cplx<double>));
  b += 2 * align16((size_t)max_nc * sizeof(cplx<double>));
  b += align16((size_t)3 * max_nc * sizeof(cplx<double>));
  b += 3 * align16(s * sizeof(cplx<double>));
  b += align16(s * sizeof(double));
  b += align16(8 * sizeof(double)) + align16(4 * sizeof(int));
  return b;
}

template <typename T, int NT>
__device__ Lds<T> carve(unsigned char* base, int max_nj, int max_nc, int maxit) {
  Lds<T> L;
  const size_t s = (size_t)maxit + 2;
  L.stride = (int)s;
  size_t o = 0;
  auto take = [&](size_t bytes) { unsigned char* p = base + o; o += align16(bytes); return p; };
  L.A = (cplx<T>*)take((size_t)max_nj * sizeof(cplx<T>));
  L.B = (cplx<T>*)take((size_t)max_nj * sizeof(cplx<T>));
  L.tab = (cplx<T>*)take(kClasses * kStencilPts * sizeof(cplx<T>));
  L.red = (cplx<T>*)take((size_t)(NT / kWave) * s * sizeof(cplx<T>));
  L.hT = (cplx<T>*)take(s * sizeof(cplx<T>));
  L.hU = (cplx<T>*)take(s * sizeof(cplx<T>));
  L.sv = (cplx<double>*)take(s * sizeof(cplx<double>));
  L.cv = (cplx<double>*)take(s * sizeof(cplx<double>));
  L.ct = (cplx<double>*)take((size_t)max_nc * sizeof(cplx<double>));
  L.ca = (cplx<double>*)take((size_t)max_nc * sizeof(cplx<double>));
  L.lc = (cplx<double>*)take((size_t)3 * max_nc * sizeof(cplx<double>));
  L.h = (cplx<double>*)take(s * sizeof(cplx<double>));
  L.g = (cplx<double>*)take(s * sizeof(cplx<double>));
  L.sn = (cplx<double>*)take(s * sizeof(cplx<double>));
  L.cs = (double*)take(s * sizeof(double));
  L.scal = (double*)take(8 * sizeof(double));
  L.ctrl = (int*)take(4 * sizeof(int));
  return L;
}

// `v` if `keep`, else 0 (a select, not a branch).
template <typename T>
__device__ __forceinline__ cplx<T> keep_or_zero(bool keep, cplx<T> v) {
  return cplx<T>{keep ? v.re : T(0), keep ? v.im : T(0)};
}

// out (=|-=) B_j in over the tile; no synchronisation.  Neighbours outside the tile are
// read at the node itself and multiplied by zero, so the seven reads of a node are issued
// together without branches (adding 0 * c leaves the sum unchanged).
template <typename T, bool kSubtract>
__device__ __forceinline__ void apply_B(const SubDesc& d, const cplx<T>* tab, const cplx<T>* in, cplx<T>* out) {
  const int nx = d.nx, ny = d.ny, nj = nx * ny;
  for (int n = threadIdx.x; n < nj; n += blockDim.x) {
    const int lj = n / nx, li = n - lj * nx;
    const cplx<T>* c = tab + kStencilPts * node_class(d.i0 + li, d.j0 + lj, d.ax, d.bx, d.ay, d.by);
    const bool hw = li > 0, he = li < nx - 1, hs = lj > 0, hn = lj < ny - 1;
    const cplx<T> xc = in[n];
    const cplx<T> xw = keep_or_zero(hw, in[hw ? n - 1 : n]);
    const cplx<T> xe = keep_or_zero(he, in[he ? n + 1 : n]);
    const cplx<T> xs = keep_or_zero(hs, in[hs ? n - nx : n]);
    const cplx<T> xsw = keep_or_zero(hs && hw, in[hs && hw ? n - nx - 1 : n]);
    const cplx<T> xn = keep_or_zero(hn, in[hn ? n + nx : n]);
    const cplx<T> xne = keep_or_zero(hn && he, in[hn && he ? n + nx + 1 : n]);
    cplx<T> acc = c[kC] * xc;
    acc = cfma(c[kW], xw, acc);
    acc = cfma(c[kE], xe, acc);
    acc = cfma(c[kS], xs, acc);
    acc = cfma(c[kSW], xsw, acc);
    acc = cfma(c[kN], xn, acc);
    acc = cfma(c[kNE], xne, acc);
    out[n] = kSubtract ? out[n] - acc : acc;
  }
}

// t = Z^T v, accumulated in double.  With `padded`, t is a coarse-solve LDS array and
// its entries from mx * my up to the solve length ncp are set to 0.
template <typename T>
__device__ __forceinline__ void restrict_to(const SubDesc& d, const cplx<T>* v, cplx<double>* t,
                                            bool padded = true) {
  const int nc = d.mx * d.my;
  if (d.defl != kLinear) {
    const int nout = padded ? d.ncp : nc;
    for (int c = threadIdx.x; c < nout; c += blockDim.x) {
      cplx<double> acc = czero<double>();
      if (c < nc) {
        const int cy = c / d.mx, cx = c - cy * d.mx;
        for (int py = max(2 * cy - 1, 0); py <= 2 * cy + 3 && py < d.ny; ++py) {
          const double wy = zweight_kind(kBezier, py, cy);
          for (int px = max(2 * cx - 1, 0); px <= 2 * cx + 3 && px < d.nx; ++px)
            acc = acc + (wy * zweight_kind(kBezier, px, cx)) * ccast<double>(v[py * d.nx + px]);
        }
      }
      t[c] = acc;
    }
    return;
  }
  // fine rows/columns 2c, 2c+1, 2c+2 with weights 1/2, 1, 1/2; only 2c+2 can fall outside
  // the tile, and is then read at 2c+1 with weight 0
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    const int cy = c / d.mx, cx = c - cy * d.mx;
    const bool xin = 2 * cx + 2 < d.nx, yin = 2 * cy + 2 < d.ny;
    const int px[3] = {2 * cx, 2 * cx + 1, xin ? 2 * cx + 2 : 2 * cx + 1};
    const int py[3] = {2 * cy, 2 * cy + 1, yin ? 2 * cy + 2 : 2 * cy + 1};
    const double wx[3] = {0.5, 1.0, xin ? 0.5 : 0.0};
    const double wy[3] = {0.5, 1.0, yin ? 0.5 : 0.0};
    cplx<T> vv[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int e = 0; e < 3; ++e) vv[b][e] = v[py[b] * d.nx + px[e]];
    cplx<double> acc = czero<double>();
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int e = 0; e < 3; ++e) acc = acc + (wy[b] * wx[e]) * ccast<double>(vv[b][e]);
    t[c] = acc;
  }
}

// Z y at fine node (li, lj).
__device__ __forceinline__ cplx<double> prolong_at(const SubDesc& d, const cplx<double>* y, int li, int lj) {
  if (d.defl != kLinear) {
    // coarse nodes within distance 2 of the fine node: c in [(i - 3) / 2, (i + 1) / 2]
    const int ca = (li - 3) >> 1, cb = (lj - 3) >> 1;
    cplx<double> acc = czero<double>();
#pragma unroll
    for (int b = cb; b <= cb + 2; ++b) {
      if (b < 0 || b >= d.my) continue;
      const double wy = zweight_kind(kBezier, lj, b);
#pragma unroll
      for (int a2 = ca; a2 <= ca + 2; ++a2) {
        if (a2 < 0 || a2 >= d.mx) continue;
        acc = acc + (wy * zweight_kind(kBezier, li, a2)) * y[b * d.mx + a2];
      }
    }
    return acc;
  }
  // coarse nodes (li - 1) >> 1 and the next one per direction; one outside the coarse grid
  // is read at a valid node with weight 0
  const int ca = (li - 1) >> 1, cb = (lj - 1) >> 1;
  double wy[2], wx[2];
  int by[2], bx[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int b = cb + q, a2 = ca + q;
    const bool yok = b >= 0 && b < d.my, xok = a2 >= 0 && a2 < d.mx;
    by[q] = yok ? b : 0;
    bx[q] = xok ? a2 : 0;
    wy[q] = yok ? zweight(lj, b) : 0.0;
    wx[q] = xok ? zweight(li, a2) : 0.0;
  }
  cplx<double> yv[2][2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int e = 0; e < 2; ++e) yv[q][e] = y[by[q] * d.mx + bx[e]];
  cplx<double> acc = czero<double>();
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int e = 0; e < 2; ++e) acc = acc + (wy[q] * wx[e]) * yv[q][e];
  return acc;
}

template <typename T>
__device__ __forceinline__ void prolong_to(const SubDesc& d, const cplx<double>* y, cplx<T>* v) {
  const int nx = d.nx, nj = nx * d.ny;
  for (int n = threadIdx.x; n < nj; n += blockDim.x) {
    const int lj = n / nx, li = n - lj * nx;
    v[n] = ccast<T>(prolong_at(d, y, li, lj));
  }
}

// B := P B A  (deflated operator applied to tile A; A is overwritten).
template <typename T, int NT>
__device__ __forceinline__ void deflated_op(const SubDesc& d, const cplx<double>* fac, Lds<T>& L) {
  apply_B<T, false>(d, L.tab, L.A, L.B);
  lds_barrier();
  restrict_to(d, L.B, L.ct);
  lds_barrier();
  coarse_solve<NT>(d, fac, L.lc, L.ct, L.ca);
  prolong_to(d, L.ca, L.A);
  lds_barrier();
  apply_B<T, true>(d, L.tab, L.A, L.B);
  lds_barrier();
}

// Workgroup sum of a real partial; every thread gets the total.
template <typename T, int NT>
__device__ __forceinline__ double block_sum(T part, Lds<T>& L) {
  part = wave_total(part);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  lds_barrier();
  if (lane == kWave - 1) L.red[wave].re = part;
  lds_barrier();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) s += (double)L.red[w].re;
  lds_barrier();
  return s;
}

template <int NT>
__device__ __forceinline__ double block_sum_f64(double part, double* red) {
  part = wave_total(part);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  lds_barrier();
  if (lane == kWave - 1) red[wave] = part;
  lds_barrier();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) s += red[w];
  lds_barrier();
  return s;
}

template <typename T, int NT>
__device__ __forceinline__ double tile_norm(const SubDesc& d, const cplx<T>* v, Lds<T>& L) {
  const int nj = d.nx * d.ny;
  T p = T(0);
  for (int n = threadIdx.x; n < nj; n += NT) p += cabs2(v[n]);
  return sqrt(block_sum<T, NT>(p, L));
}

// Gram-Schmidt coefficients against V[0..k]: red[w * S + i] = wave w's partial of
// conj(V_i) . B for i <= k, and red[w * S + k + 1] = wave w's partial of |B|^2 when
// with_norm.  The basis is swept kDotChunk vectors at a time and each thread loads the
// chunk's entries of kSweepNodes nodes at once (indices clamped to valid vectors and nodes,
// surplus products multiplied by zero), so that many loads are in flight per wave: the
// sweeps are bound by how many bytes a CU has in flight, not by arithmetic.  Each
// thread's partial sums still add its nodes in increasing order.
constexpr int kDotChunk = 8;
constexpr int kSweepNodes = 1;   // 2 and 4 measured slower over the whole kernel (register pressure)
template <typename T, int NT>
__device__ __forceinline__ void basis_dots(const cplx<T>* __restrict__ V, int nj, int k, const cplx<T>* B,
                                           cplx<T>* red, int S, bool with_norm) {
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  for (int i0 = 0; i0 <= k; i0 += kDotChunk) {
    cplx<T> acc[kDotChunk];
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) acc[q] = czero<T>();
    for (int n0 = tid; n0 < nj; n0 += kSweepNodes * NT) {
      int nn[kSweepNodes];
      cplx<T> w[kSweepNodes];
#pragma unroll
      for (int e = 0; e < kSweepNodes; ++e) {
        const int n = n0 + e * NT;
        nn[e] = n < nj ? n : n0;
        w[e] = keep_or_zero(n < nj, B[nn[e]]);
      }
      cplx<T> v[kSweepNodes][kDotChunk];
#pragma unroll
      for (int e = 0; e < kSweepNodes; ++e)
#pragma unroll
        for (int q = 0; q < kDotChunk; ++q) v[e][q] = V[(long long)min(i0 + q, k) * nj + nn[e]];
#pragma unroll
      for (int e = 0; e < kSweepNodes; ++e)
#pragma unroll
        for (int q = 0; q < kDotChunk; ++q)
          if (i0 + q <= k) acc[q] = acc[q] + cmulc(v[e][q], w[e]);
    }
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) {
      if (i0 + q <= k) {
        cplx<T> p = acc[q];
        p.re = wave_total(p.re);
        p.im = wave_total(p.im);
        if (lane == kWave - 1) red[wave * S + i0 + q] = p;
      }
    }
  }
  if (with_norm) {
    T q = T(0);
    for (int n = tid; n < nj; n += NT) q += cabs2(B[n]);
    q = wave_total(q);
    if (lane == kWave - 1) red[wave * S + k + 1] = cplx<T>{q, T(0)};
  }
}

// B[n] (+|-)= sum_{i < cnt} V_i[n] c_i over the tile, chunked like basis_dots: every load
// of a chunk and of the thread's kSweepNodes nodes is issued before the first product
// (indices past cnt are clamped to a valid vector and their coefficient skipped).
constexpr int kUpdChunk = 8;
template <typename T, int NT, bool kSubtract>
__device__ __forceinline__ void basis_combine(const cplx<T>* __restrict__ V, int nj, int cnt, const cplx<T>* c,
                                              cplx<T>* B) {
  if (cnt <= 0) return;
  for (int n0 = threadIdx.x; n0 < nj; n0 += kSweepNodes * NT) {
    int nn[kSweepNodes];
    cplx<T> acc[kSweepNodes];
#pragma unroll
    for (int e = 0; e < kSweepNodes; ++e) {
      const int n = n0 + e * NT;
      nn[e] = n < nj ? n : n0;
      acc[e] = B[nn[e]];
    }
    for (int i0 = 0; i0 < cnt; i0 += kUpdChunk) {
      cplx<T> v[kSweepNodes][kUpdChunk];
#pragma unroll
      for (int e = 0; e < kSweepNodes; ++e)
#pragma unroll
        for (int q = 0; q < kUpdChunk; ++q) v[e][q] = V[(long long)min(i0 + q, cnt - 1) * nj + nn[e]];
#pragma unroll
      for (int e = 0; e < kSweepNodes; ++e)
#pragma unroll
        for (int q = 0; q < kUpdChunk; ++q)
          if (i0 + q < cnt) acc[e] = kSubtract ? acc[e] - v[e][q] * c[i0 + q] : acc[e] + v[e][q] * c[i0 + q];
    }
#pragma unroll
    for (int e = 0; e < kSweepNodes; ++e)
      if (n0 + e * NT < nj) B[n0 + e * NT] = acc[e];
  }
}

// Delayed-CGS2 update sweep: with u = u~_j in slot j of V and w in LDS, at every node
//   v_j     = u / alpha - sum_{i<j} V_i ca_i              (written to slot j, over u)
//   u~_{j+1} = (w - sum_{i<j} V_i cb_i - u e) / gamma      (written to slot j + 1 and the tile)
// one load of each basis entry for both outputs, chunked like basis_combine.
template <typename T, int NT>
__device__ __forceinline__ void basis_update2(cplx<T>* V, int nj, int j, const cplx<T>* ca, const cplx<T>* cb,
                                              T inv_alpha, cplx<T> e, T inv_gamma, const cplx<T>* w,
                                              cplx<T>* tile) {
  cplx<T>* Vj = V + (long long)j * nj;
  cplx<T>* Vn = Vj + nj;
  for (int n = threadIdx.x; n < nj; n += NT) {
    const cplx<T> uo = Vj[n], wn = w[n];
    cplx<T> aa = czero<T>(), ab = czero<T>();
    for (int i0 = 0; i0 < j; i0 += kUpdChunk) {
      cplx<T> v[kUpdChunk];
#pragma unroll
      for (int q = 0; q < kUpdChunk; ++q) v[q] = V[(long long)min(i0 + q, j - 1) * nj + n];
#pragma unroll
      for (int q = 0; q < kUpdChunk; ++q) {
        if (i0 + q < j) {
          aa = cfma(v[q], ca[i0 + q], aa);
          ab = cfma(v[q], cb[i0 + q], ab);
        }
      }
    }
    const cplx<T> un = inv_gamma * (wn - ab - uo * e);
    Vj[n] = inv_alpha * uo - aa;
    Vn[n] = un;
    tile[n] = un;
  }
}

template <typename T>
__host__ __device__ constexpr double breakdown_eps() { return sizeof(T) == 4 ? 4e-6 : 1e-14; }

}  // namespace

// A value every lane holds alike (a workgroup sum read back from LDS), moved to scalar
// registers: the Krylov loop keeps such values live, and in vector registers they would
// push the coarse solve's factor ring into scratch.
__device__ __forceinline__ double uniform_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT) inner_solve_kernel(InnerArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int sidx = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
  const int nsub = a.cs.nsub;
  const int rhs = sidx / nsub, sub = sidx - rhs * nsub;
  if (a.done && a.done[rhs]) return;
  const SubDesc d = a.subs[sub];
  Lds<T> L = carve<T, NT>(smem, a.max_nj, a.max_nc, a.maxit);
  const int tid = threadIdx.x;
  const int nx = d.nx, nj = d.nx * d.ny;
  const int maxit = a.maxit;
  const long long fo = (long long)rhs * a.nfine + d.off;
  cplx<T>* F = a.F + fo;
  cplx<T>* W = a.W + fo;
  cplx<T>* X = a.X + fo;
  cplx<T>* V = a.V + fo * (maxit + 1);
  // R factor of the rotated Hessenberg matrix, then T (candidates in the orthonormal basis),
  // each maxit x maxit with column c at c * maxit
  cplx<double>* R = a.R + (long long)sidx * 2 * maxit * maxit;
  cplx<double>* Tm = R + (long long)maxit * maxit;
  // coarse vectors kept for the recovery: slot 0 E^{-1} Z^T f, slot 1 E^{-1} Z^T B x0, slot 2 + i
  // E^{-1} Z^T B u~_i (written and read back by the same thread for each entry)
  cplx<double>* Sc = a.Sc ? a.Sc + (long long)sidx * (maxit + 2) * a.max_nc : nullptr;
  auto keep_coarse = [&](int slot) {
    if (Sc)
      for (int e = tid; e < d.ncp; e += NT) Sc[(long long)slot * a.max_nc + e] = L.ca[e];
  };
  const int ldg = a.cs.n - 1;
  const long long jstep = a.jdev ? (long long)*a.jdev : 0;
  const cplx<double>* __restrict__ rin = a.r ? a.r + jstep * a.rslot : nullptr;
  cplx<double>* __restrict__ zout = a.z ? a.z + jstep * a.zslot : nullptr;

  build_class_table<T>(d.robin, a.cs.kh, a.cs.kh2, L.tab);
  stage_lower(d, a.Ec, L.lc);
  // Gather f = R_j r.  The local system is linear and its stopping test relative,
  // so it is solved for f / ||f|| (norm taken in FP64) and the solution rescaled:
  // local right-hand sides far from the sources are many orders of magnitude below
  // 1 and would lose precision, or underflow, in complex64.
  double fn2 = 0.0;
  for (int n = tid; n < nj; n += NT) {
    if (rin) {
      const int lj = n / nx, li = n - lj * nx;
      fn2 += cabs2(rin[(long long)rhs * a.rstride + (long long)(d.j0 + lj - 1) * ldg + (d.i0 + li - 1)]);
    } else {
      fn2 += cabs2(ccast<double>(F[n]));
    }
  }
  const double fnorm = uniform_f64(sqrt(block_sum_f64<NT>(fn2, (double*)L.red)));
  const double fscale = fnorm > 0.0 ? 1.0 / fnorm : 0.0;
  // F holds the scaled right-hand side when gathered here; a caller-supplied F is
  // left untouched and scaled on use (fmul).
  const T fmul = rin ? T(1) : T(fscale);
  for (int n = tid; n < nj; n += NT) {
    cplx<T> v;
    if (rin) {
      const int lj = n / nx, li = n - lj * nx;
      v = ccast<T>(fscale * rin[(long long)rhs * a.rstride + (long long)(d.j0 + lj - 1) * ldg + (d.i0 + li - 1)]);
      F[n] = v;
    } else {
      v = fmul * F[n];
    }
    L.B[n] = v;
  }
  lds_barrier();
  // P f = f - B Z E^{-1} Z^T f   (tile B)
  restrict_to(d, L.B, L.ct);
  lds_barrier();
  coarse_solve<NT>(d, a.fac, L.lc, L.ct, L.ca);
  keep_coarse(0);
  prolong_to(d, L.ca, L.A);
  lds_barrier();
  apply_B<T, true>(d, L.tab, L.A, L.B);
  lds_barrier();
  const double ref = uniform_f64(tile_norm<T, NT>(d, L.B, L));

  bool accepted = false;
  const bool offered = ref > 0.0 && (a.guess || a.gtile);
  int k = 0;
  bool converged = true;
  if (ref > 0.0) {
    if (a.guess || a.gtile) {
      // the solve runs on f / ||f||: a packed guess is scaled by 1 / ||f||, a network
      // tile (scaled by sqrt(n_j) / ||f||) by 1 / sqrt(n_j)
      const cplx<T>* gs = a.guess ? a.guess + fo : nullptr;
      const float* gt = a.gtile ? a.gtile + (size_t)sidx * a.gT * a.gT * 2 : nullptr;
      const T gmul = gt ? T(1.0 / sqrt((double)nj)) : T(fscale);
      for (int n = tid; n < nj; n += NT) {
        W[n] = L.B[n];
        cplx<T> gv;
        if (gt) {
          const int lj = n / nx, li = n - lj * nx;
          const float* q = gt + ((size_t)lj * a.gT + li) * 2;
          gv = cplx<T>{gmul * T(q[0]), gmul * T(q[1])};
        } else {
          gv = gmul * gs[n];
        }
        L.A[n] = gv;
        X[n] = gv;
      }
      lds_barrier();
      deflated_op<T, NT>(d, a.fac, L);   // tile B = P B g
      keep_coarse(1);
      for (int n = tid; n < nj; n += NT) L.B[n] = W[n] - L.B[n];
      lds_barrier();
      const double rn = tile_norm<T, NT>(d, L.B, L);
      accepted = __builtin_amdgcn_readfirstlane(rn < ref ? 1 : 0) != 0;
      if (!accepted) {
        for (int n = tid; n < nj; n += NT) L.B[n] = W[n];
        lds_barrier();
      }
    }
    const double beta = accepted ? tile_norm<T, NT>(d, L.B, L) : ref;
    converged = beta <= a.tol * ref;
    if (!converged) {
      // candidate u~_0 = r0 / beta in slot 0 and tile A
      const T inv = T(1.0 / beta);
      for (int n = tid; n < nj; n += NT) {
        const cplx<T> v = inv * L.B[n];
        V[n] = v;
        L.A[n] = v;
      }
      if (tid == 0) {
        L.g[0] = cplx<double>{beta, 0.0};
        L.ctrl[0] = 0;
      }
      __syncthreads();
    }
    const int S = L.stride;
    // Iteration j: (1) s = V_j^H u~_j, nu = |u~_j|^2, alpha = sqrt(nu - |s|^2); column j-1 of
    // H becomes final (tentative column + gamma_j s, subdiagonal gamma_j alpha), is rotated,
    // and the residual estimate decides convergence before the operator is applied;
    // (2) w = P B u~_j; (3) c = V_j^H w, mu = u~_j^H w, omega = |w|^2; tentative column j:
    // c and h_jj = (mu - s^H c) / alpha; gamma_{j+1} from Pythagoras (a scale only: the
    // next step's nu corrects it exactly); (4) one update sweep writes v_j and u~_{j+1}.
    int j = 0;
    while (!converged) {
      basis_dots<T, NT>(V, nj, j - 1, L.A, L.red, S, true);
      lds_barrier();
      for (int i = tid; i <= j; i += NT) {
        cplx<double> sacc = czero<double>();
#pragma unroll
        for (int w = 0; w < NT / kWave; ++w) sacc = sacc + ccast<double>(L.red[w * S + i]);
        L.sv[i] = sacc;
      }
      lds_barrier();
      if (tid == 0) {
        double ss = 0.0;
        for (int i = 0; i < j; ++i) ss += cabs2(L.sv[i]);
        const double nu = L.sv[j].re;
        const double a2 = nu - ss, afloor = 1e-30 * (nu > 0.0 ? nu : 1.0);
        const double alpha = sqrt(a2 > afloor ? a2 : afloor);
        L.scal[0] = 1.0 / alpha;
        L.scal[1] = alpha;
        if (j == 0) {
          L.g[0] = alpha * L.g[0];
        } else {
          const int c0 = j - 1;
          cplx<double>* col = L.h;
          const double gm = L.scal[3];
          for (int i = 0; i <= c0; ++i) col[i] = col[i] + gm * L.sv[i];
          for (int i = 0; i < c0; ++i) {
            const cplx<double> x0 = col[i], x1 = col[i + 1];
            col[i] = L.cs[i] * x0 + L.sn[i] * x1;
            col[i + 1] = L.cs[i] * x1 - cplx<double>{L.sn[i].re, -L.sn[i].im} * x0;
          }
          const double hnext = gm * alpha;
          const cplx<double> av = col[c0];
          const double aa = sqrt(cabs2(av));
          double c;
          cplx<double> sv, r;
          if (hnext == 0.0) {
            c = 1.0; sv = czero<double>(); r = av;
          } else if (aa == 0.0) {
            c = 0.0; sv = cplx<double>{1.0, 0.0}; r = cplx<double>{hnext, 0.0};
          } else {
            const double t = hypot(aa, hnext);
            const cplx<double> ph = cplx<double>{av.re / aa, av.im / aa};
            c = aa / t;
            sv = (hnext / t) * ph;
            r = t * ph;
          }
          L.cs[c0] = c;
          L.sn[c0] = sv;
          col[c0] = r;
          for (int i = 0; i <= c0; ++i) R[(long long)c0 * maxit + i] = col[i];
          const cplx<double> gk = L.g[c0];
          L.g[c0 + 1] = czero<double>() - cplx<double>{sv.re, -sv.im} * gk;
          L.g[c0] = c * gk;
          const double res = sqrt(cabs2(L.g[c0 + 1]));
          const bool brk = hnext <= breakdown_eps<T>() * L.scal[2];
          L.ctrl[0] = (res <= a.tol * ref || brk) ? 1 : 0;
        }
      }
      lds_barrier();
      converged = __builtin_amdgcn_readfirstlane(L.ctrl[0]) != 0;
      if (converged || j == maxit) break;
      {
        // column j of T and the update coefficients of v_j
        const double inv_alpha = L.scal[0];
        cplx<double>* Tc = Tm + (long long)j * maxit;
        for (int i = tid; i <= j; i += NT) {
          Tc[i] = i < j ? L.sv[i] : cplx<double>{L.scal[1], 0.0};
          if (i < j) L.hT[i] = ccast<T>(inv_alpha * L.sv[i]);
        }
      }
      deflated_op<T, NT>(d, a.fac, L);   // tile B = w = P B u~_j (tile A overwritten)
      keep_coarse(2 + j);
      basis_dots<T, NT>(V, nj, j, L.B, L.red, S, true);
      lds_barrier();
      for (int i = tid; i <= j + 1; i += NT) {
        cplx<double> sacc = czero<double>();
#pragma unroll
        for (int w = 0; w < NT / kWave; ++w) sacc = sacc + ccast<double>(L.red[w * S + i]);
        L.cv[i] = sacc;
      }
      lds_barrier();
      if (tid == 0) {
        cplx<double> sTc = czero<double>();
        double cc = 0.0;
        for (int i = 0; i < j; ++i) {
          sTc = sTc + cmulc(L.sv[i], L.cv[i]);
          cc += cabs2(L.cv[i]);
        }
        const double inv_alpha = L.scal[0];
        const cplx<double> hjj = inv_alpha * (L.cv[j] - sTc);
        const double om = L.cv[j + 1].re;
        double g2 = om - cc - cabs2(hjj);
        const double gfloor = 1e-28 * (om > 0.0 ? om : 1.0);
        if (!(g2 > gfloor)) g2 = gfloor;
        const double gm = sqrt(g2);
        for (int i = 0; i < j; ++i) L.h[i] = L.cv[i];
        L.h[j] = hjj;
        const cplx<double> e = inv_alpha * hjj;
        L.scal[2] = sqrt(om > 0.0 ? om : 0.0);   // ||w||: breakdown scale of column j
        L.scal[3] = gm;
        L.scal[4] = 1.0 / gm;
        L.scal[6] = e.re;
        L.scal[7] = e.im;
      }
      lds_barrier();
      const cplx<double> e{L.scal[6], L.scal[7]};
      for (int i = tid; i < j; i += NT) L.hU[i] = ccast<T>(L.cv[i] - L.sv[i] * e);
      lds_barrier();
      basis_update2<T, NT>(V, nj, j, L.hT, L.hU, T(L.scal[0]), ccast<T>(e), T(L.scal[4]), L.B, L.A);
      __syncthreads();
      ++j;
    }
    k = j;
    // y = R^{-1} g (upper triangular, k x k).  R is copied into the free tile A first when
    // it fits (all threads load it side by side), so the serial substitution reads LDS.
    const bool r_lds = (size_t)k * k * sizeof(cplx<double>) <= (size_t)a.max_nj * sizeof(cplx<T>);
    cplx<double>* Rl = reinterpret_cast<cplx<double>*>(L.A);
    if (r_lds) {
      __syncthreads();   // thread 0's global stores of R are visible to the workgroup
      for (int e = tid; e < k * k; e += NT) {
        const int j = e / k, i = e - j * k;
        if (i <= j) Rl[e] = R[(long long)j * maxit + i];
      }
      lds_barrier();
    }
    if (tid == 0) {
      for (int i = k - 1; i >= 0; --i) {
        cplx<double> sacc = L.g[i];
        for (int j = i + 1; j < k; ++j)
          sacc = sacc - (r_lds ? Rl[j * k + i] : R[(long long)j * maxit + i]) * L.h[j];
        L.h[i] = sacc * cinv(r_lds ? Rl[i * k + i] : R[(long long)i * maxit + i]);
      }
    }
    lds_barrier();
    // x coefficients in the orthonormal basis: T y (T upper triangular)
    for (int i = tid; i < k; i += NT) {
      cplx<double> acc = czero<double>();
      for (int l = i; l < k; ++l) acc = acc + Tm[(long long)l * maxit + i] * L.h[l];
      L.hT[i] = ccast<T>(acc);
    }
    lds_barrier();
  }
  // x = x0 + V y   (tile A)
  for (int n = tid; n < nj; n += NT) L.A[n] = accepted ? X[n] : czero<T>();
  basis_combine<T, NT, false>(V, nj, k, L.hT, L.A);
  lds_barrier();
  // recovery: u = x + Z E^{-1} Z^T (f - B x)
  if (Sc) {
    // from the kept coarse vectors (y_i in L.h)
    for (int e = tid; e < d.ncp; e += NT) {
      cplx<double> c = Sc[e];
      if (accepted) c = c - Sc[a.max_nc + e];
      for (int i0 = 0; i0 < k; i0 += kUpdChunk) {
        cplx<double> sv[kUpdChunk];
#pragma unroll
        for (int q = 0; q < kUpdChunk; ++q) sv[q] = Sc[(long long)(2 + min(i0 + q, k - 1)) * a.max_nc + e];
#pragma unroll
        for (int q = 0; q < kUpdChunk; ++q)
          if (i0 + q < k) c = c - L.h[i0 + q] * sv[q];
      }
      L.ca[e] = c;
    }
    lds_barrier();
  } else {
    const int ny = d.ny;
    for (int n = tid; n < nj; n += NT) {
      const int lj = n / nx, li = n - lj * nx;
      const cplx<T>* c = L.tab + kStencilPts * node_class(d.i0 + li, d.j0 + lj, d.ax, d.bx, d.ay, d.by);
      cplx<T> acc = c[kC] * L.A[n];
      if (li > 0) acc = cfma(c[kW], L.A[n - 1], acc);
      if (li < nx - 1) acc = cfma(c[kE], L.A[n + 1], acc);
      if (lj > 0) {
        acc = cfma(c[kS], L.A[n - nx], acc);
        if (li > 0) acc = cfma(c[kSW], L.A[n - nx - 1], acc);
      }
      if (lj < ny - 1) {
        acc = cfma(c[kN], L.A[n + nx], acc);
        if (li < nx - 1) acc = cfma(c[kNE], L.A[n + nx + 1], acc);
      }
      L.B[n] = fmul * F[n] - acc;
    }
    lds_barrier();
    restrict_to(d, L.B, L.ct);
    lds_barrier();
    coarse_solve<NT>(d, a.fac, L.lc, L.ct, L.ca);
  }
  for (int n = tid; n < nj; n += NT) {
    const int lj = n / nx, li = n - lj * nx;
    const cplx<T> u = L.A[n] + ccast<T>(prolong_at(d, L.ca, li, lj));
    if (a.U) a.U[fo + n] = ccast<T>(fnorm * ccast<double>(u));
    if (zout) {
      const int gi = d.i0 + li, gj = d.j0 + lj;
      if (gi >= d.oi0 && gi <= d.oi1 && gj >= d.oj0 && gj <= d.oj1) {
        const long long gidx = (long long)(gj - 1) * ldg + (gi - 1);
        const cplx<double> add = a.zadd ? a.zadd[(long long)rhs * a.ndof + gidx] : czero<double>();
        zout[(long long)rhs * a.zstride + gidx] = fnorm * ccast<double>(u) + add;
      }
    }
  }
  if (tid == 0) {
    if (a.iters) a.iters[sidx] = k;
    if (a.flags) a.flags[sidx] = (accepted ? 1 : 0) | (converged ? 0 : 2);
    if (a.counters) {
      atomicAdd(a.counters + 0, (unsigned long long)k);
      atomicAdd(a.counters + 1, 1ull);
      atomicMax(a.counters + 2, (unsigned long long)k);
      if (accepted) atomicAdd(a.counters + 3, 1ull);
      const unsigned long long s = sizeof(cplx<T>), nn = (unsigned long long)nj, kk = (unsigned long long)k;
      const unsigned long long own = (unsigned long long)(d.oi1 - d.oi0 + 1) * (d.oj1 - d.oj0 + 1);
      const unsigned long long fac_bytes = 16ull * (unsigned long long)coarse_solve_values(d);
      const unsigned long long ncp = (unsigned long long)d.ncp;
      unsigned long long bytes = 16ull * nn + (a.zadd ? 32ull : 16ull) * own +
                                 (Sc ? (kk + 1) * fac_bytes + 16ull * ncp * (2 * kk + 2) : (kk + 2) * fac_bytes) +
                                 (kk ? s * nn * (1 + 3 * kk + 3 * kk * (kk + 1) / 2) : 0ull) + 2 * s * nn;
      if (offered) bytes += fac_bytes + (a.gtile ? 8ull : s) * nn + 3 * s * nn + (Sc ? 32ull * ncp : 0ull);
      atomicAdd(a.counters + 4, bytes);
    }
  }
}

template <typename T>
size_t inner_lds_bytes(int max_nj, int max_nc, int maxit) {
  return std::max(lds_bytes<T>(max_nj, max_nc, maxit, kInnerThreads), lds_bytes<T>(max_nj, max_nc, maxit, 256));
}

template <typename T>
hipError_t launch_inner_solve(const InnerArgs<T>& a, hipStream_t st) {
  const int nblocks = a.cs.nsub * a.nrhs;
  if (a.nt == 256) {
    const size_t lds = lds_bytes<T>(a.max_nj, a.max_nc, a.maxit, 256);
    hipLaunchKernelGGL((inner_solve_kernel<T, 256>), dim3(nblocks), dim3(256), lds, st, a);
  } else {
    const size_t lds = lds_bytes<T>(a.max_nj, a.max_nc, a.maxit, kInnerThreads);
    hipLaunchKernelGGL((inner_solve_kernel<T, kInnerThreads>), dim3(nblocks), dim3(kInnerThreads), lds, st, a);
  }
  return hipGetLastError();
}

// ---- kernel-level operations on packed vectors ---------------------------------------

template <typename T>
__global__ void __launch_bounds__(kBlock) local_apply_kernel(const SubDesc* __restrict__ subs, Consts cs,
                                                              const cplx<T>* __restrict__ v,
                                                              cplx<T>* __restrict__ w) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SubDesc d = subs[blockIdx.x];
  cplx<T>* tab = (cplx<T>*)smem;
  cplx<T>* tile = (cplx<T>*)(smem + align16(kClasses * kStencilPts * sizeof(cplx<T>)));
  build_class_table<T>(d.robin, cs.kh, cs.kh2, tab);
  const int nj = d.nx * d.ny;
  for (int n = threadIdx.x; n < nj; n += blockDim.x) tile[n] = v[d.off + n];
  __syncthreads();
  apply_B<T, false>(d, tab, tile, w + d.off);
}

template <typename T>
hipError_t launch_local_apply(const SubDesc* subs, int nsub, Consts cs, int, const cplx<T>* v, cplx<T>* w,
                              int max_nj, hipStream_t st) {
  const size_t lds = align16(kClasses * kStencilPts * sizeof(cplx<T>)) + (size_t)max_nj * sizeof(cplx<T>);
  hipLaunchKernelGGL(local_apply_kernel<T>, dim3(nsub), dim3(kBlock), lds, st, subs, cs, v, w);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) deflated_apply_kernel(const SubDesc* __restrict__ subs, Consts cs,
                                                                 const cplx<double>* __restrict__ fac,
                                                                 const cplx<double>* __restrict__ Ec,
                                                                 const cplx<T>* __restrict__ v,
                                                                 cplx<T>* __restrict__ w, int max_nj, int max_nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SubDesc d = subs[blockIdx.x];
  Lds<T> L = carve<T, kBlock>(smem, max_nj, max_nc, 1);
  build_class_table<T>(d.robin, cs.kh, cs.kh2, L.tab);
  stage_lower(d, Ec, L.lc);
  const int nj = d.nx * d.ny;
  for (int n = threadIdx.x; n < nj; n += blockDim.x) L.A[n] = v[d.off + n];
  __syncthreads();
  deflated_op<T, kBlock>(d, fac, L);
  for (int n = threadIdx.x; n < nj; n += blockDim.x) w[d.off + n] = L.B[n];
}

template <typename T>
hipError_t launch_deflated_apply(const SubDesc* subs, int nsub, Consts cs, int, const cplx<double>* fac,
                                 const cplx<double>* Ec, const cplx<T>* v, cplx<T>* w, int max_nj, int max_nc,
                                 hipStream_t st) {
  const size_t lds = lds_bytes<T>(max_nj, max_nc, 1, kBlock);
  hipLaunchKernelGGL(deflated_apply_kernel<T>, dim3(nsub), dim3(kBlock), lds, st, subs, cs, fac, Ec, v, w,
                     max_nj, max_nc);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) restrict_kernel(const SubDesc* __restrict__ subs,
                                                           const cplx<double>* __restrict__ v,
                                                           cplx<double>* __restrict__ t) {
  const SubDesc d = subs[blockIdx.x];
  restrict_to(d, v + d.off, t + d.coff, false);
}

hipError_t launch_restrict(const SubDesc* subs, int nsub, const cplx<double>* v, cplx<double>* t,
                           hipStream_t st) {
  hipLaunchKernelGGL(restrict_kernel, dim3(nsub), dim3(kBlock), 0, st, subs, v, t);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) prolong_kernel(const SubDesc* __restrict__ subs,
                                                          const cplx<double>* __restrict__ y,
                                                          cplx<double>* __restrict__ v) {
  const SubDesc d = subs[blockIdx.x];
  prolong_to(d, y + d.coff, v + d.off);
}

hipError_t launch_prolong(const SubDesc* subs, int nsub, const cplx<double>* y, cplx<double>* v,
                          hipStream_t st) {
  hipLaunchKernelGGL(prolong_kernel, dim3(nsub), dim3(kBlock), 0, st, subs, y, v);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) coarse_solve_kernel(const SubDesc* __restrict__ subs,
                                                               const cplx<double>* __restrict__ fac,
                                                               const cplx<double>* __restrict__ Ec,
                                                               const cplx<double>* __restrict__ t,
                                                               cplx<double>* __restrict__ y, int max_nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SubDesc d = subs[blockIdx.x];
  cplx<double>* ct = (cplx<double>*)smem;
  cplx<double>* ca = ct + max_nc;
  cplx<double>* lc = ca + max_nc;
  const int nc = d.mx * d.my;
  for (int c = threadIdx.x; c < d.ncp; c += blockDim.x) ct[c] = c < nc ? t[d.coff + c] : czero<double>();
  stage_lower(d, Ec, lc);
  __syncthreads();
  coarse_solve<kBlock>(d, fac, lc, ct, ca);
  for (int c = threadIdx.x; c < nc; c += blockDim.x) y[d.coff + c] = ca[c];
}

hipError_t launch_coarse_solve(const SubDesc* subs, int nsub, const cplx<double>* fac, const cplx<double>* Ec,
                               const cplx<double>* t, cplx<double>* y, int max_nc, hipStream_t st) {
  const size_t lds = 5 * (size_t)max_nc * sizeof(cplx<double>);
  hipLaunchKernelGGL(coarse_solve_kernel, dim3(nsub), dim3(kBlock), lds, st, subs, fac, Ec, t, y, max_nc);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) gather_kernel(const SubDesc* __restrict__ subs, Consts cs,
                                                         const cplx<double>* __restrict__ r,
                                                         cplx<T>* __restrict__ f, long long nfine,
                                                         long long ndof) {
  const SubDesc d = subs[blockIdx.x];
  const int rhs = blockIdx.y, nj = d.nx * d.ny, ldg = cs.n - 1;
  for (int n = threadIdx.x; n < nj; n += blockDim.x) {
    const int lj = n / d.nx, li = n - lj * d.nx;
    f[rhs * nfine + d.off + n] =
        ccast<T>(r[rhs * ndof + (long long)(d.j0 + lj - 1) * ldg + (d.i0 + li - 1)]);
  }
}

template <typename T>
hipError_t launch_gather(const SubDesc* subs, int nsub, Consts cs, const cplx<double>* r, cplx<T>* f,
                         long long nfine, long long ndof, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(gather_kernel<T>, dim3(nsub, nrhs), dim3(kBlock), 0, st, subs, cs, r, f, nfine, ndof);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) scatter_kernel(const SubDesc* __restrict__ subs, Consts cs,
                                                          const cplx<T>* __restrict__ u,
                                                          cplx<double>* __restrict__ z, long long nfine,
                                                          long long ndof) {
  const SubDesc d = subs[blockIdx.x];
  const int rhs = blockIdx.y, ldg = cs.n - 1;
  const int ow = d.oi1 - d.oi0 + 1, oh = d.oj1 - d.oj0 + 1;
  for (int n = threadIdx.x; n < ow * oh; n += blockDim.x) {
    const int gj = d.oj0 + n / ow, gi = d.oi0 + n % ow;
    const int li = gi - d.i0, lj = gj - d.j0;
    z[rhs * ndof + (long long)(gj - 1) * ldg + (gi - 1)] = ccast<double>(u[rhs * nfine + d.off + lj * d.nx + li]);
  }
}

template <typename T>
hipError_t launch_scatter(const SubDesc* subs, int nsub, Consts cs, const cplx<T>* u, cplx<double>* z,
                          long long nfine, long long ndof, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(scatter_kernel<T>, dim3(nsub, nrhs), dim3(kBlock), 0, st, subs, cs, u, z, nfine, ndof);
  return hipGetLastError();
}

template <typename T>
hipError_t configure_inner(int max_nj, int max_nc, int maxit) {
  int dev = 0, maxlds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  // A kernel whose LDS at these sizes exceeds the device limit is left unconfigured: set-up
  // has already rejected the handle unless it never launches that kernel (exact local solves
  // do not run the subdomain GMRES), and a launch of it is refused by the runtime.
  auto set = [&](const void* fn, size_t lds) {
    if (e == hipSuccess && lds > 65536 && lds <= (size_t)maxlds)
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  };
  set((const void*)inner_solve_kernel<T, kInnerThreads>, lds_bytes<T>(max_nj, max_nc, maxit, kInnerThreads));
  set((const void*)inner_solve_kernel<T, 256>, lds_bytes<T>(max_nj, max_nc, maxit, 256));
  set((const void*)deflated_apply_kernel<T>, lds_bytes<T>(max_nj, max_nc, 1, kBlock));
  set((const void*)local_apply_kernel<T>,
      align16(kClasses * kStencilPts * sizeof(cplx<T>)) + (size_t)max_nj * sizeof(cplx<T>));
  set((const void*)coarse_solve_kernel, 5 * (size_t)max_nc * sizeof(cplx<double>));
  return e;
}

#define DDH_INSTANTIATE(T)                                                                                   \
  template hipError_t launch_inner_solve<T>(const InnerArgs<T>&, hipStream_t);                                \
  template hipError_t configure_inner<T>(int, int, int);                                                     \
  template size_t inner_lds_bytes<T>(int, int, int);                                                          \
  template hipError_t launch_local_apply<T>(const SubDesc*, int, Consts, int, const cplx<T>*, cplx<T>*, int,  \
                                            hipStream_t);                                                     \
  template hipError_t launch_deflated_apply<T>(const SubDesc*, int, Consts, int, const cplx<double>*,         \
                                               const cplx<double>*, const cplx<T>*, cplx<T>*, int, int,       \
                                               hipStream_t);                                                  \
  template hipError_t launch_gather<T>(const SubDesc*, int, Consts, const cplx<double>*, cplx<T>*, long long, \
                                       long long, int, hipStream_t);                                          \
  template hipError_t launch_scatter<T>(const SubDesc*, int, Consts, const cplx<T>*, cplx<double>*, long long, \
                                        long long, int, hipStream_t);

DDH_INSTANTIATE(float)
DDH_INSTANTIATE(double)

}  // namespace ddh
