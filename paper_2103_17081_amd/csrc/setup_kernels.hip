// Set-up kernels: Galerkin coarse matrices E_j = Z_j^T B_j Z_j and their FP64
// block factorisations (see coarse.hpp).  One workgroup per subdomain.
#include "coarse.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace ddh {

// Stencil point offsets in the order of StencilPoint.
__constant__ int kSx[kStencilPts] = {0, -1, 1, 0, 0, -1, 1};
__constant__ int kSy[kStencilPts] = {0, 0, 0, -1, 1, -1, 1};

// E(c, c+d) = sum_p Z(p, c) sum_q B(p, q) Z(q, c+d), p over the support of Z_c
// (3 x 3 fine nodes for linear deflation, 5 x 5 for Bezier); coarse_coefs(kind) values
// per coarse node.
__global__ void __launch_bounds__(kBlock) assemble_coarse_kernel(const SubDesc* __restrict__ subs, Consts cs,
                                                                  int local_bc, cplx<double>* __restrict__ Ec) {
  const SubDesc d = subs[blockIdx.x];
  __shared__ cplx<double> tab[kClasses * kStencilPts];
  build_class_table<double>(d.robin, cs.kh, cs.kh2, tab);
  __syncthreads();
  const int kind = d.defl, R = zreach(kind), W = 2 * R + 1, K = W * W;
  const int nc = d.mx * d.my;
  for (int e = threadIdx.x; e < nc * K; e += blockDim.x) {
    const int c = e / K, o = e % K;
    const int cx = c % d.mx, cy = c / d.mx;
    const int qx = cx + o % W - R, qy = cy + o / W - R;
    cplx<double> acc = czero<double>();
    if (qx >= 0 && qx < d.mx && qy >= 0 && qy < d.my) {
      for (int py = max(2 * cy + 1 - R, 0); py <= 2 * cy + 1 + R && py < d.ny; ++py) {
        for (int px = max(2 * cx + 1 - R, 0); px <= 2 * cx + 1 + R && px < d.nx; ++px) {
          const double wz = zweight_kind(kind, px, cx) * zweight_kind(kind, py, cy);
          const int cls = local_bc == 0 ? node_class(d.i0 + px, d.j0 + py, d.ax, d.bx, d.ay, d.by) : 4;
          for (int s = 0; s < kStencilPts; ++s) {
            const int fx = px + kSx[s], fy = py + kSy[s];
            if (fx < 0 || fx >= d.nx || fy < 0 || fy >= d.ny) continue;
            const double wq = zweight_kind(kind, fx, qx) * zweight_kind(kind, fy, qy);
            if (wq != 0.0) acc = acc + (wz * wq) * tab[cls * kStencilPts + s];
          }
        }
      }
    }
    Ec[(d.coff + c) * K + o] = acc;
  }
}

// Largest |entry| among n complex coefficients, workgroup-cooperative (every thread gets it):
// the scale that the pivot magnitudes of a factorisation are compared against.
__device__ double block_absmax(const cplx<double>* __restrict__ c, long long n, double* sh) {
  double m = 0.0;
  for (long long e = threadIdx.x; e < n; e += blockDim.x) m = fmax(m, sqrt(cabs2(c[e])));
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, kWave));
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = m;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) r = fmax(r, sh[w]);
  __syncthreads();
  return r;
}

// In-place Gauss-Jordan inverse with partial pivoting of the n x n row-major matrix
// A (global memory; element (r, c) at r*n + c), workgroup-cooperative.  Returns the
// smallest |pivot| met.
__device__ double gauss_jordan_inverse(cplx<double>* A, int n, int* perm, cplx<double>* colp,
                                       double* sh_pivabs) {
  const int tid = threadIdx.x;
  double minpiv = 1e300;
  for (int p = 0; p < n; ++p) {
    if (tid == 0) {
      int q = p;
      double best = cabs2(A[p * n + p]);
      for (int r = p + 1; r < n; ++r) {
        const double v = cabs2(A[r * n + p]);
        if (v > best) { best = v; q = r; }
      }
      perm[p] = q;
      *sh_pivabs = sqrt(best);
    }
    __syncthreads();
    const int q = perm[p];
    if (q != p) {
      for (int c = tid; c < n; c += blockDim.x) {
        const cplx<double> x = A[p * n + c];
        A[p * n + c] = A[q * n + c];
        A[q * n + c] = x;
      }
    }
    __syncthreads();
    minpiv = fmin(minpiv, *sh_pivabs);
    const cplx<double> inv = cinv(A[p * n + p]);
    __syncthreads();
    // scale row p (the pivot entry becomes 1/pivot) and stash column p
    for (int c = tid; c < n; c += blockDim.x) A[p * n + c] = (c == p) ? inv : inv * A[p * n + c];
    for (int r = tid; r < n; r += blockDim.x) colp[r] = A[r * n + p];
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int r = e / n, c = e - r * n;
      if (r == p) continue;
      const cplx<double> f = colp[r];
      A[r * n + c] = (c == p) ? czero<double>() - A[p * n + p] * f : A[r * n + c] - A[p * n + c] * f;
    }
    __syncthreads();
  }
  // undo the row interchanges by swapping columns in reverse order
  for (int p = n - 1; p >= 0; --p) {
    const int q = perm[p];
    if (q != p) {
      for (int r = tid; r < n; r += blockDim.x) {
        const cplx<double> x = A[r * n + p];
        A[r * n + p] = A[r * n + q];
        A[r * n + q] = x;
      }
    }
    __syncthreads();
  }
  return minpiv;
}

// Twisted block factorisation of E (linear deflation; layout and relations in
// coarse.hpp).  D_i from the stored own-row couplings, L_i from the stored lower
// couplings, U_i = L_{i+1}^T.
__global__ void __launch_bounds__(kBlock) factor_coarse_twisted_kernel(const SubDesc* __restrict__ subs,
                                                                        const cplx<double>* __restrict__ Ec,
                                                                        cplx<double>* __restrict__ fac,
                                                                        double* __restrict__ pivmin) {
  const SubDesc d = subs[blockIdx.x];
  __shared__ int perm[kMaxMx];
  __shared__ cplx<double> colp[kMaxMx];
  __shared__ double pivabs;
  const int mx = d.mx, my = d.my, mm = mx * mx, tid = threadIdx.x, p = twist_row(my);
  const cplx<double>* ec = Ec + d.coff * 9;
  cplx<double>* F = fac + d.goff;
  // D_i(r, c), L_i(r, c) (unknown r of row i to unknown c of row i-1), U_i(r, c) = L_{i+1}(c, r)
  auto Dv = [&](int i, int r, int c) {
    return (c - r >= -1 && c - r <= 1) ? ec[(size_t)(i * mx + r) * 9 + 4 + (c - r)] : czero<double>();
  };
  auto Lv = [&](int i, int r, int c) {
    return (c - r >= -1 && c - r <= 1) ? ec[(size_t)(i * mx + r) * 9 + 1 + (c - r)] : czero<double>();
  };
  auto Uv = [&](int i, int r, int c) { return Lv(i + 1, c, r); };
  auto blk = [&](int b) { return F + (size_t)b * mm; };
  double minp = 1e300;
  // top: G_i = (D_i - L_i H_{i-1})^{-1}, H_i = G_i U_i
  for (int i = 0; i < p; ++i) {
    cplx<double>* G = blk(tw_G(i));
    for (int e = tid; e < mm; e += blockDim.x) {
      const int r = e / mx, c = e - r * mx;
      cplx<double> s = Dv(i, r, c);
      if (i > 0) {
        const cplx<double>* Hp = blk(tw_H(p, i - 1));
        for (int rr = max(r - 1, 0); rr <= min(r + 1, mx - 1); ++rr) s = s - Lv(i, r, rr) * Hp[rr * mx + c];
      }
      G[e] = s;
    }
    __syncthreads();
    minp = fmin(minp, gauss_jordan_inverse(G, mx, perm, colp, &pivabs));
    cplx<double>* H = blk(tw_H(p, i));
    for (int e = tid; e < mm; e += blockDim.x) {
      const int r = e / mx, c = e - r * mx;
      cplx<double> s = czero<double>();
      for (int cc = max(c - 1, 0); cc <= min(c + 1, mx - 1); ++cc) s = s + G[r * mx + cc] * Uv(i, cc, c);
      H[e] = s;
    }
    __syncthreads();
  }
  // bottom: K_i = (D_i - U_i J_{i+1})^{-1}, J_i = K_i L_i
  for (int i = my - 1; i > p; --i) {
    cplx<double>* K = blk(tw_K(p, i));
    for (int e = tid; e < mm; e += blockDim.x) {
      const int r = e / mx, c = e - r * mx;
      cplx<double> s = Dv(i, r, c);
      if (i < my - 1) {
        const cplx<double>* Jn = blk(tw_J(my, i + 1));
        for (int rr = max(r - 1, 0); rr <= min(r + 1, mx - 1); ++rr) s = s - Uv(i, r, rr) * Jn[rr * mx + c];
      }
      K[e] = s;
    }
    __syncthreads();
    minp = fmin(minp, gauss_jordan_inverse(K, mx, perm, colp, &pivabs));
    cplx<double>* J = blk(tw_J(my, i));
    for (int e = tid; e < mm; e += blockDim.x) {
      const int r = e / mx, c = e - r * mx;
      cplx<double> s = czero<double>();
      for (int cc = max(c - 1, 0); cc <= min(c + 1, mx - 1); ++cc) s = s + K[r * mx + cc] * Lv(i, cc, c);
      J[e] = s;
    }
    __syncthreads();
  }
  // middle: M = (D_p - L_p H_{p-1} - U_p J_{p+1})^{-1}
  cplx<double>* M = blk(tw_M(my));
  for (int e = tid; e < mm; e += blockDim.x) {
    const int r = e / mx, c = e - r * mx;
    cplx<double> s = Dv(p, r, c);
    for (int rr = max(r - 1, 0); rr <= min(r + 1, mx - 1); ++rr) {
      if (p > 0) s = s - Lv(p, r, rr) * blk(tw_H(p, p - 1))[rr * mx + c];
      if (p < my - 1) s = s - Uv(p, r, rr) * blk(tw_J(my, p + 1))[rr * mx + c];
    }
    M[e] = s;
  }
  __syncthreads();
  minp = fmin(minp, gauss_jordan_inverse(M, mx, perm, colp, &pivabs));
  __shared__ double red[kBlock / kWave];
  const double emax = block_absmax(ec, (long long)mx * my * 9, red);
  if (tid == 0) {
    pivmin[2 * blockIdx.x] = minp;
    pivmin[2 * blockIdx.x + 1] = emax;
  }
}

hipError_t launch_factor_coarse_twisted(const SubDesc* subs, int nsub, const cplx<double>* Ec, cplx<double>* fac,
                                        double* pivmin, hipStream_t st) {
  hipLaunchKernelGGL(factor_coarse_twisted_kernel, dim3(nsub), dim3(kBlock), 0, st, subs, Ec, fac, pivmin);
  return hipGetLastError();
}

// Block LU over pairs of coarse rows (Bezier deflation, see coarse.hpp).  Unknown k of
// block row I is coarse node (k % mx, 2 I + k / mx); a row beyond my is an identity row.
__device__ __forceinline__ cplx<double> paired_coef(const SubDesc& d, const cplx<double>* __restrict__ ec, int I,
                                                    int k, int J, int kk) {
  const int x = k % d.mx, y = 2 * I + k / d.mx;
  const int xx = kk % d.mx, yy = 2 * J + kk / d.mx;
  if (y >= d.my || yy >= d.my) return (y == yy && x == xx) ? cplx<double>{1.0, 0.0} : czero<double>();
  const int dx = xx - x, dy = yy - y;
  if (dx < -2 || dx > 2 || dy < -2 || dy > 2) return czero<double>();
  return ec[(size_t)(y * d.mx + x) * 25 + 5 * (dy + 2) + (dx + 2)];
}

__global__ void __launch_bounds__(kBlock) factor_coarse_paired_kernel(const SubDesc* __restrict__ subs,
                                                                       const cplx<double>* __restrict__ Ec,
                                                                       cplx<double>* __restrict__ fac,
                                                                       double* __restrict__ pivmin) {
  const SubDesc d = subs[blockIdx.x];
  __shared__ int perm[kMaxMx];
  __shared__ cplx<double> colp[kMaxMx];
  __shared__ double pivabs;
  const int bm = d.bmx, bn = d.bmy, mm = bm * bm, tid = threadIdx.x;
  const cplx<double>* ec = Ec + d.coff * 25;
  cplx<double>* F = fac + d.goff;
  double minp = 1e300;
  for (int I = 0; I < bn; ++I) {
    cplx<double>* G = F + (size_t)I * mm;
    cplx<double>* Lb = F + (size_t)(2 * bn - 2 + I) * mm;   // L_I (I >= 1)
    const cplx<double>* Hprev = F + (size_t)(bn + I - 1) * mm;
    if (I > 0) {
      for (int e = tid; e < mm; e += blockDim.x) Lb[e] = paired_coef(d, ec, I, e / bm, I - 1, e % bm);
      __syncthreads();
    }
    // S_I = D_I - L_I H_{I-1}
    for (int e = tid; e < mm; e += blockDim.x) {
      const int r = e / bm, c = e - r * bm;
      cplx<double> s = paired_coef(d, ec, I, r, I, c);
      if (I > 0)
        for (int k = 0; k < bm; ++k) s = s - Lb[r * bm + k] * Hprev[k * bm + c];
      G[e] = s;
    }
    __syncthreads();
    minp = fmin(minp, gauss_jordan_inverse(G, bm, perm, colp, &pivabs));
    if (I < bn - 1) {
      // H_I = G_I U_I
      cplx<double>* H = F + (size_t)(bn + I) * mm;
      for (int e = tid; e < mm; e += blockDim.x) {
        const int r = e / bm, c = e - r * bm;
        cplx<double> s = czero<double>();
        for (int k = 0; k < bm; ++k) s = s + G[r * bm + k] * paired_coef(d, ec, I, k, I + 1, c);
        H[e] = s;
      }
    }
    __syncthreads();
  }
  __shared__ double red[kBlock / kWave];
  const double emax = block_absmax(ec, (long long)d.mx * d.my * 25, red);
  if (tid == 0) {
    pivmin[2 * blockIdx.x] = minp;
    pivmin[2 * blockIdx.x + 1] = emax;
  }
}

hipError_t launch_factor_coarse_paired(const SubDesc* subs, int nsub, const cplx<double>* Ec, cplx<double>* fac,
                                       double* pivmin, hipStream_t st) {
  hipLaunchKernelGGL(factor_coarse_paired_kernel, dim3(nsub), dim3(kBlock), 0, st, subs, Ec, fac, pivmin);
  return hipGetLastError();
}

hipError_t launch_assemble_coarse(const SubDesc* subs, int nsub, Consts cs, int local_bc, cplx<double>* Ec,
                                  hipStream_t st) {
  hipLaunchKernelGGL(assemble_coarse_kernel, dim3(nsub), dim3(kBlock), 0, st, subs, cs, local_bc, Ec);
  return hipGetLastError();
}


}  // namespace ddh
