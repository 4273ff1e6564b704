// Coarse deflation operator E = Z^T B Z (Sec. 2, eq. 4) for linear interpolation
// Z = Z^y kron Z^x (eq. 5), and its FP64 block LU.
//
// With coarse nodes ordered x fastest, E couples a coarse node only to its 3 x 3
// coarse neighbours, so E is block tridiagonal in the coarse rows: diagonal blocks
// D_i, sub-diagonal L_i (row i to row i-1), super-diagonal U_i (row i to row i+1),
// each an mx x mx tridiagonal matrix.  Block LU without block pivoting:
//     S_0 = D_0,  G_i = S_i^{-1},  H_i = G_i U_i,  S_{i+1} = D_{i+1} - L_{i+1} H_i.
// Solve E y = t:  a_0 = G_0 t_0,  a_i = G_i (t_i - L_i a_{i-1});
//                 y_{my-1} = a_{my-1},  y_i = a_i - H_i y_{i+1}.
// Each S_i is inverted by Gauss-Jordan elimination with partial pivoting.  The
// solve is then 2 my - 1 dense mx x mx products instead of the n_c-step scalar
// recurrences of a banded triangular solve; it streams the same number of bytes.
//
// Storage per subdomain at SubDesc::goff (complex<double>): the my blocks G_i, then
// the my-1 blocks H_i, each mx*mx column-major (element (r, c) at c*mx + r).
// E itself is kept as nine coefficients per coarse node, offset index
// o = 3*(dy+1) + (dx+1) for the neighbour (cx+dx, cy+dy).
#pragma once

#include "common.hpp"

namespace ddh {

constexpr int kMaxMx = 128;   // largest coarse block (mx) the kernels support

__host__ __device__ __forceinline__ long long coarse_factor_size(int mx, int my) {
  return (long long)(2 * my - 1) * mx * mx;
}

// y = E^{-1} t for one subdomain, workgroup-cooperative.  `t` and `a` live in LDS
// (n_c entries each, may not alias); the result overwrites `a`.  `tmp` holds mx
// entries of LDS.  All threads of the workgroup must call it.
__device__ __forceinline__ void coarse_solve(const SubDesc& d, const cplx<double>* __restrict__ fac,
                                             const cplx<double>* __restrict__ Ec,
                                             const cplx<double>* t, cplx<double>* a,
                                             cplx<double>* tmp) {
  const int mx = d.mx, my = d.my, tid = threadIdx.x;
  const int mm = mx * mx;
  const cplx<double>* ec = Ec + d.coff * 9;
  fac += d.goff;
  for (int i = 0; i < my; ++i) {
    for (int r = tid; r < mx; r += blockDim.x) {
      cplx<double> s = t[i * mx + r];
      if (i > 0) {
        const cplx<double>* row = ec + (size_t)(i * mx + r) * 9;   // dy = -1: o = 0, 1, 2
#pragma unroll
        for (int dr = -1; dr <= 1; ++dr) {
          int c = r + dr;
          if (c >= 0 && c < mx) s = s - row[dr + 1] * a[(i - 1) * mx + c];
        }
      }
      tmp[r] = s;
    }
    __syncthreads();
    const cplx<double>* G = fac + (size_t)i * mm;
    for (int r = tid; r < mx; r += blockDim.x) {
      cplx<double> s = czero<double>();
      for (int c = 0; c < mx; ++c) s = cfma(G[c * mx + r], tmp[c], s);
      a[i * mx + r] = s;
    }
    __syncthreads();
  }
  for (int i = my - 2; i >= 0; --i) {
    const cplx<double>* H = fac + (size_t)(my + i) * mm;
    for (int r = tid; r < mx; r += blockDim.x) {
      cplx<double> s = a[i * mx + r];
      for (int c = 0; c < mx; ++c) s = s - H[c * mx + r] * a[(i + 1) * mx + c];
      a[i * mx + r] = s;
    }
    __syncthreads();
  }
}

}  // namespace ddh
