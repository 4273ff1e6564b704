// Shared device/host definitions of the ddhelm HIP library (gfx950 / CDNA4).
//
// Complex numbers are interleaved (re, im) pairs, the layout of complex64 /
// complex128 torch tensors.  Fine-level Krylov work runs in the template scalar T
// (float for the mixed-precision inner solver, double for the all-FP64 one);
// the coarse deflation solve and the outer FGMRES always run in double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddh {

constexpr int kBlock = 256;        // threads per workgroup of the kernel-level subdomain operations
constexpr int kInnerThreads = 512; // threads per workgroup of the batched subdomain-solve kernel
constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kWavesPerBlock = kBlock / kWave;

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc + a * b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
template <typename T>
__host__ __device__ __forceinline__ T cabs2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename D, typename S>
__host__ __device__ __forceinline__ cplx<D> ccast(cplx<S> a) { return {(D)a.re, (D)a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> czero() { return {T(0), T(0)}; }
// 1 / a
__host__ __device__ __forceinline__ cplx<double> cinv(cplx<double> a) {
  double d = 1.0 / (a.re * a.re + a.im * a.im);
  return {a.re * d, -a.im * d};
}

// Load of a complex<double> that the caller streams once (the outer basis in the dot and
// update sweeps): the non-temporal hint keeps it from displacing reused lines in the
// caches, worth about 6% of sweep bandwidth on gfx950.
__device__ __forceinline__ cplx<double> load_stream(const cplx<double>* p) {
  const double* q = reinterpret_cast<const double*>(p);
  return cplx<double>{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
}

// Geometry of one overlapping subdomain and its packed storage.
//
// The subdomain is the node rectangle [ax, bx] x [ay, by] (its cells are
// [ax, bx) x [ay, by)).  Its local unknowns form the tile of nx * ny nodes
// starting at global node (i0, j0), x fastest.  Nodes (i, j) with
// oi0 <= i <= oi1 and oj0 <= j <= oj1 are owned (Boolean partition of unity).
// Bit s of `robin` is set when side s (0 left, 1 right, 2 bottom, 3 top) carries
// the impedance condition.
struct SubDesc {
  int i0, j0, nx, ny;
  int ax, bx, ay, by;
  int oi0, oi1, oj0, oj1;
  int mx, my;        // coarse grid mx * my (coarse node c on fine node 2c + 1 per direction)
  int robin;
  int defl;          // deflation vectors: 0 linear interpolation, 1 quadratic Bezier
  int bmx, bmy;      // block factorisation of E: bmy block rows of bmx unknowns (linear: mx, my;
                     // Bezier: pairs of coarse rows, 2 mx and ceil(my / 2))
  int ncp;           // coarse vector length of the solve, bmx * bmy (>= mx * my)
  int pad;
  long long off;     // offset of the tile in packed fine vectors (elements)
  long long coff;    // offset in packed coarse vectors (elements)
  long long goff;    // offset of the coarse factors (complex<double> elements)
};

// Problem-wide constants.
struct Consts {
  int n;             // intervals per edge; interior nodes 1..n-1
  int nsub;
  double k, h, kh, kh2;
};

// Seven-point stencil of one row class.  Order: centre, W, E, S, N, SW, NE.
// (NW and SE couplings vanish for the SW->NE cell diagonal.)
constexpr int kStencilPts = 7;
constexpr int kClasses = 9;        // (left edge | middle | right edge) x (bottom | middle | top)

// Workgroup barrier for phases that exchange data only through LDS: waits for this
// wave's LDS operations, not for its outstanding global loads (which __syncthreads'
// fence would drain), so loads issued ahead of the barrier stay in flight.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---- wavefront / workgroup reductions ------------------------------------
// DPP row operations (16-lane rows): swap adjacent lanes, swap lane pairs, mirror
// within each half row, mirror within the row.  Applied in this order with adds,
// every lane of a row ends with the sum over its 16 lanes (over 8 after three).
constexpr int kDppXor1 = 0xB1;          // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;   // row_half_mirror
constexpr int kDppMirror = 0x140;       // row_mirror

constexpr int kDppBcast15 = 0x142;      // row_bcast:15 (last lane of each row to the next row)
constexpr int kDppBcast31 = 0x143;      // row_bcast:31 (lane 31 to rows 2 and 3)

// DPP move of v; rows outside RowMask read 0.
template <int Ctrl, int RowMask = 0xF>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, RowMask, 0xF, false));
}
template <int Ctrl, int RowMask = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), Ctrl, RowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), Ctrl, RowMask, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int Ctrl, int RowMask = 0xF>
__device__ __forceinline__ float dpp(float v) { return dpp_f32<Ctrl, RowMask>(v); }
template <int Ctrl, int RowMask = 0xF>
__device__ __forceinline__ double dpp(double v) { return dpp_f64<Ctrl, RowMask>(v); }

// Sum over each aligned group of `Lanes` (2, 4, 8 or 16) lanes; all lanes get it.
template <int Lanes, typename T>
__device__ __forceinline__ T row_sum(T v) {
  static_assert(Lanes == 2 || Lanes == 4 || Lanes == 8 || Lanes == 16, "row_sum group size");
  v += dpp<kDppXor1>(v);
  if (Lanes >= 4) v += dpp<kDppXor2>(v);
  if (Lanes >= 8) v += dpp<kDppHalfMirror>(v);
  if (Lanes >= 16) v += dpp<kDppMirror>(v);
  return v;
}

// Sum over the whole wavefront, valid in its last lane only: the 16-lane row sums, then
// row 1 (3) adds the last lane of row 0 (2), then rows 2 and 3 add lane 31.  VALU only:
// no LDS crossbar traffic, unlike the shuffle butterfly of wave_sum.
template <typename T>
__device__ __forceinline__ T wave_total(T v) {
  v = row_sum<16>(v);
  v += dpp<kDppBcast15, 0xA>(v);
  v += dpp<kDppBcast31, 0xC>(v);
  return v;
}

// Sum over the whole wavefront; every lane gets it.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

}  // namespace ddh
