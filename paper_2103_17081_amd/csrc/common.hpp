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

constexpr int kBlock = 256;        // threads per workgroup of the subdomain kernels
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
  int mx, my;        // coarse grid mx * my (linear deflation, H = 2h)
  int robin;
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

// ---- wavefront / workgroup reductions ------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

}  // namespace ddh
