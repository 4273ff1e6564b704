// Matrix-free P1 Helmholtz rows (Sec. 2, eq. 2) on a uniform mesh whose cells are
// split along the SW->NE diagonal.
//
// A row is the sum of the contributions of the cells around its node that lie in
// the (sub)domain.  Per cell, with kh2 = (k h)^2, stiffness K and mass M of the two
// P1 triangles give (node -> neighbour):
//   node at the cell's SW corner: centre 1 - kh2/6,  E and N: -1/2 - kh2/24,  NE: -kh2/12
//   node at the cell's SE corner: centre 1 - kh2/12, W and N: -1/2 - kh2/24
//   node at the cell's NE corner: centre 1 - kh2/6,  W and S: -1/2 - kh2/24,  SW: -kh2/12
//   node at the cell's NW corner: centre 1 - kh2/12, E and S: -1/2 - kh2/24
// (the corner names are those of the cell; the node's neighbours are listed from
// the node).  The impedance condition d_n u - i k u = 0 on an interface side adds
// -i k (h/6)[2 1; 1 2] per boundary segment: -i kh/3 to the centre and -i kh/6 to
// the neighbour along the side.  Interior rows reduce to the classic stencil:
// centre 4 - kh2/2, E/W/N/S -1 - kh2/12, NE/SW -kh2/12.
//
// Which cells exist depends only on whether the node lies on the subdomain's left
// or right side and bottom or top side, so every subdomain has nine row classes.
#pragma once

#include "common.hpp"

namespace ddh {

enum StencilPoint { kC = 0, kW = 1, kE = 2, kS = 3, kN = 4, kSW = 5, kNE = 6 };

// Row class of node (i, j): 3 * ycls + xcls with cls 0 on the low side, 2 on the
// high side, 1 elsewhere.
__host__ __device__ __forceinline__ int node_class(int i, int j, int ax, int bx, int ay, int by) {
  int xc = (i == ax) ? 0 : ((i == bx) ? 2 : 1);
  int yc = (j == ay) ? 0 : ((j == by) ? 2 : 1);
  return 3 * yc + xc;
}

// Coefficients of row class `cls` for a subdomain whose impedance sides are `robin`.
__host__ __device__ inline void class_stencil(int cls, int robin, double kh, double kh2,
                                              cplx<double> out[kStencilPts]) {
  const int xc = cls % 3, yc = cls / 3;
  const bool onL = xc == 0, onR = xc == 2, onB = yc == 0, onT = yc == 2;
  double re[kStencilPts] = {0, 0, 0, 0, 0, 0, 0};
  double im[kStencilPts] = {0, 0, 0, 0, 0, 0, 0};
  const double side = -0.5 - kh2 / 24.0;
  if (!onR && !onT) { re[kC] += 1.0 - kh2 / 6.0;  re[kE] += side; re[kN] += side; re[kNE] += -kh2 / 12.0; }
  if (!onL && !onT) { re[kC] += 1.0 - kh2 / 12.0; re[kW] += side; re[kN] += side; }
  if (!onL && !onB) { re[kC] += 1.0 - kh2 / 6.0;  re[kW] += side; re[kS] += side; re[kSW] += -kh2 / 12.0; }
  if (!onR && !onB) { re[kC] += 1.0 - kh2 / 12.0; re[kE] += side; re[kS] += side; }
  const double cdiag = -kh / 3.0, coff = -kh / 6.0;
  // vertical sides: segments towards N (if not on top) and S (if not on bottom)
  if ((onL && (robin & 1)) || (onR && (robin & 2))) {
    if (!onT) { im[kC] += cdiag; im[kN] += coff; }
    if (!onB) { im[kC] += cdiag; im[kS] += coff; }
  }
  // horizontal sides: segments towards E (if not on the right) and W (if not on the left)
  if ((onB && (robin & 4)) || (onT && (robin & 8))) {
    if (!onR) { im[kC] += cdiag; im[kE] += coff; }
    if (!onL) { im[kC] += cdiag; im[kW] += coff; }
  }
  for (int p = 0; p < kStencilPts; ++p) out[p] = cplx<double>{re[p], im[p]};
}

// Fill a 9 x 7 class table (workgroup-cooperative: threads 0..8 each fill a class).
template <typename T>
__device__ __forceinline__ void build_class_table(int robin, double kh, double kh2, cplx<T>* tab) {
  const int t = threadIdx.x;
  if (t < kClasses) {
    cplx<double> c[kStencilPts];
    class_stencil(t, robin, kh, kh2, c);
#pragma unroll
    for (int p = 0; p < kStencilPts; ++p) tab[t * kStencilPts + p] = ccast<T>(c[p]);
  }
}

// Linear-interpolation weight of fine node `i` for coarse node `c` (H = 2h, coarse
// node c sits on fine node 2c+1): 1 at distance 0, 1/2 at distance 1.
__host__ __device__ __forceinline__ double zweight(int i, int c) {
  int d = i - (2 * c + 1);
  return d == 0 ? 1.0 : ((d == 1 || d == -1) ? 0.5 : 0.0);
}

// Deflation vectors per direction (Sec. 2, eq. 5): linear interpolation, or the
// quadratic rational Bezier stencil 1/8 [1 4 6 4 1] centred on fine node 2c+1 (the
// printed map from fine to coarse values, read as Z^T).  zreach: largest distance from
// 2c+1 with a non-zero weight, which is also the coupling radius of E = Z^T B Z.
enum DeflationKind { kLinear = 0, kBezier = 1 };
__host__ __device__ __forceinline__ int zreach(int kind) { return kind == kBezier ? 2 : 1; }
__host__ __device__ __forceinline__ double zweight_kind(int kind, int i, int c) {
  int d = i - (2 * c + 1);
  d = d < 0 ? -d : d;
  if (kind == kBezier) return d == 0 ? 0.75 : (d == 1 ? 0.5 : (d == 2 ? 0.125 : 0.0));
  return d == 0 ? 1.0 : (d == 1 ? 0.5 : 0.0);
}
// Coefficients of E stored per coarse node: (2 zreach + 1)^2, neighbour (cx+dx, cy+dy) at
// (2 zreach + 1)(dy + zreach) + (dx + zreach).
__host__ __device__ __forceinline__ int coarse_coefs(int kind) {
  const int w = 2 * zreach(kind) + 1;
  return w * w;
}

}  // namespace ddh
