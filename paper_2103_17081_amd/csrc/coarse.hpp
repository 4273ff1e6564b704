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
// the my-1 blocks H_i, each mx*mx row-major (element (r, c) at r*mx + c).
// E itself is kept as nine coefficients per coarse node, offset index
// o = 3*(dy+1) + (dx+1) for the neighbour (cx+dx, cy+dy).
#pragma once

#include "common.hpp"

namespace ddh {

constexpr int kMaxMx = 128;   // largest coarse block (mx) the kernels support
constexpr int kCoarseBatch = 8;     // block steps whose factor entries are loaded together

__host__ __device__ __forceinline__ long long coarse_factor_size(int mx, int my) {
  return (long long)(2 * my - 1) * mx * mx;
}

// Bezier deflation couples coarse nodes up to two rows apart, so its E is taken as
// block tridiagonal over pairs of coarse rows (block size bmx = 2 mx, bmy block rows; an
// odd last row is padded with an identity row).  Its factors: G_0..G_{bmy-1},
// H_0..H_{bmy-2}, then the dense lower couplings L_1..L_{bmy-1}, each bmx x bmx
// row-major.  The solve is a_I = G_I (t_I - L_I a_{I-1}), y_I = a_I - H_I y_{I+1}.
__host__ __device__ __forceinline__ long long coarse_factor_size_paired(int bmx, int bmy) {
  return (long long)(3 * bmy - 2) * bmx * bmx;
}

// Factor entries (complex<double>) one coarse solve of subdomain d reads, plus the
// staged lower couplings of E for linear deflation.
__host__ __device__ __forceinline__ long long coarse_solve_values(const SubDesc& d) {
  return d.defl == 0 ? coarse_factor_size(d.mx, d.my) + 3LL * d.mx * d.my
                     : coarse_factor_size_paired(d.bmx, d.bmy);
}

// Lanes per block row in the coarse solve: the largest power of two up to 16 with
// lanes * mx <= NT.
template <int NT>
__host__ __device__ __forceinline__ int coarse_group_lanes(int mx) {
  int l = 1;
  while (l < 16 && 2 * l * mx <= NT) l *= 2;
  return l;
}

// Copy the three lower couplings of every coarse node of E (neighbours (cx-1..cx+1,
// cy-1), offsets o = 0, 1, 2) into LDS: lc[3 c + e].  Workgroup-cooperative; the
// caller synchronises before the first coarse_solve.
__device__ __forceinline__ void stage_lower(const SubDesc& d, const cplx<double>* __restrict__ Ec,
                                            cplx<double>* lc) {
  if (d.defl != 0) return;   // the paired (Bezier) solve keeps its couplings with the factors
  const int nc = d.mx * d.my;
  const cplx<double>* ec = Ec + d.coff * 9;
  for (int e = threadIdx.x; e < 3 * nc; e += blockDim.x) lc[e] = ec[(size_t)(e / 3) * 9 + e % 3];
}

namespace detail {

// Block-tridiagonal solve with inverted diagonal blocks (the factor layout above), for
// any operator whose lower coupling L_i is tridiagonal: lower(i, c, e) is the coupling
// of unknown c of block row i to unknown c + e - 1 of block row i - 1 (e = 0, 1, 2).
// Lane l of group r owns columns c = l + q L (q < Q).  The factor entries of Depth
// consecutive steps are loaded together, in straight-line code with clamped indices,
// before those steps run, so memory latency is paid once per batch rather than once per
// step.  The coupled right-hand side t_i - L_i a_{i-1} is formed once per column
// (threads 0..mx-1, in place in t) between the block products instead of by every row
// group.
template <int L, int Q, int Depth, typename Lower>
__device__ __forceinline__ void block_solve_ring(int mx, int my, const cplx<double>* __restrict__ F, Lower lower,
                                                 cplx<double>* t, cplx<double>* a) {
  const int mm = mx * mx;
  const int r = threadIdx.x / L, l = threadIdx.x % L;
  const bool active = r < mx;
  int col[Q];
  bool ok[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    col[q] = l + q * L;
    ok[q] = active && col[q] < mx;
  }
  // element offset of this lane's entry q inside a block (clamped to 0 when unused)
  int eoff[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) eoff[q] = ok[q] ? r * mx + col[q] : 0;
  cplx<double> ring[Depth][Q];
  // forward: a_i = G_i (t_i - L_i a_{i-1}), G_i = block i
  for (int i0 = 0; i0 < my; i0 += Depth) {
#pragma unroll
    for (int u = 0; u < Depth; ++u) {
      const int blk = min(i0 + u, my - 1);
#pragma unroll
      for (int q = 0; q < Q; ++q) ring[u][q] = F[(size_t)blk * mm + eoff[q]];
    }
#pragma unroll
    for (int u = 0; u < Depth; ++u) {
      const int i = i0 + u;
      if (i < my) {
        cplx<double> acc = czero<double>();
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (ok[q]) acc = cfma(ring[u][q], t[i * mx + col[q]], acc);
        acc.re = row_sum<L>(acc.re);
        acc.im = row_sum<L>(acc.im);
        if (active && l == 0) a[i * mx + r] = acc;
        lds_barrier();
        if (i + 1 < my) {
          const int c = threadIdx.x;
          if (c < mx) {
            const cplx<double>* ap = a + i * mx + c;
            cplx<double> rhs = t[(i + 1) * mx + c] - lower(i + 1, c, 1) * ap[0];
            if (c > 0) rhs = rhs - lower(i + 1, c, 0) * ap[-1];
            if (c < mx - 1) rhs = rhs - lower(i + 1, c, 2) * ap[1];
            t[(i + 1) * mx + c] = rhs;
          }
          lds_barrier();
        }
      }
    }
  }
  // backward: y_i = a_i - H_i y_{i+1}, H_i = block my + i, i = my-2 .. 0
  for (int i0 = my - 2; i0 >= 0; i0 -= Depth) {
#pragma unroll
    for (int u = 0; u < Depth; ++u) {
      const int blk = my + max(i0 - u, 0);
#pragma unroll
      for (int q = 0; q < Q; ++q) ring[u][q] = F[(size_t)blk * mm + eoff[q]];
    }
#pragma unroll
    for (int u = 0; u < Depth; ++u) {
      const int i = i0 - u;
      if (i >= 0) {
        cplx<double> acc = czero<double>();
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (ok[q]) acc = cfma(ring[u][q], a[(i + 1) * mx + col[q]], acc);
        acc.re = row_sum<L>(acc.re);
        acc.im = row_sum<L>(acc.im);
        if (active && l == 0) a[i * mx + r] = a[i * mx + r] - acc;
        lds_barrier();
      }
    }
  }
}

// Coarse solve through the ring with E's lower couplings staged in LDS (lc).
template <int L, int Q>
__device__ __forceinline__ void coarse_solve_ring(const SubDesc& d, const cplx<double>* __restrict__ F,
                                                  const cplx<double>* lc, cplx<double>* t, cplx<double>* a) {
  auto lower = [lc, mx = d.mx](int i, int c, int e) { return lc[3 * (i * mx + c) + e]; };
  block_solve_ring<L, Q, kCoarseBatch>(d.mx, d.my, F, lower, t, a);
}

// General path for any mx <= kMaxMx: no prefetch, shuffle reductions over groups of
// L lanes (lower couplings as in block_solve_ring).
template <int NT, typename Lower>
__device__ __forceinline__ void block_solve_plain(int mx, int my, const cplx<double>* __restrict__ F, Lower lower,
                                                  cplx<double>* t, cplx<double>* a) {
  const int mm = mx * mx;
  const int L = coarse_group_lanes<NT>(mx);
  const int r = threadIdx.x / L, l = threadIdx.x % L;
  const bool active = r < mx;
  auto gsum = [&](cplx<double> v) {
    for (int o = L >> 1; o > 0; o >>= 1) {
      v.re += __shfl_xor(v.re, o, kWave);
      v.im += __shfl_xor(v.im, o, kWave);
    }
    return v;
  };
  for (int i = 0; i < my; ++i) {
    cplx<double> acc = czero<double>();
    if (active) {
      for (int c = l; c < mx; c += L) {
        cplx<double> rhs = t[i * mx + c];
        if (i > 0) {
          for (int e = 0; e < 3; ++e) {
            const int cc = c + e - 1;
            if (cc >= 0 && cc < mx) rhs = rhs - lower(i, c, e) * a[(i - 1) * mx + cc];
          }
        }
        acc = cfma(F[(size_t)i * mm + r * mx + c], rhs, acc);
      }
    }
    acc = gsum(acc);
    if (active && l == 0) a[i * mx + r] = acc;
    lds_barrier();
  }
  for (int i = my - 2; i >= 0; --i) {
    cplx<double> acc = czero<double>();
    if (active)
      for (int c = l; c < mx; c += L) acc = cfma(F[(size_t)(my + i) * mm + r * mx + c], a[(i + 1) * mx + c], acc);
    acc = gsum(acc);
    if (active && l == 0) a[i * mx + r] = a[i * mx + r] - acc;
    lds_barrier();
  }
}

template <int NT>
__device__ __forceinline__ void coarse_solve_plain(const SubDesc& d, const cplx<double>* __restrict__ F,
                                                   const cplx<double>* lc, cplx<double>* t, cplx<double>* a) {
  auto lower = [lc, mx = d.mx](int i, int c, int e) { return lc[3 * (i * mx + c) + e]; };
  block_solve_plain<NT>(d.mx, d.my, F, lower, t, a);
}

// Paired-row (Bezier) block solve with dense lower couplings; shuffle reductions over
// groups of L lanes, one LDS barrier per block product.
template <int NT>
__device__ __forceinline__ void coarse_solve_paired(const SubDesc& d, const cplx<double>* __restrict__ F,
                                                    cplx<double>* t, cplx<double>* a) {
  const int bm = d.bmx, bn = d.bmy, mm = bm * bm;
  const int L = coarse_group_lanes<NT>(bm);
  const int r = threadIdx.x / L, l = threadIdx.x % L;
  const bool active = r < bm;
  auto gsum = [&](cplx<double> v) {
    for (int o = L >> 1; o > 0; o >>= 1) {
      v.re += __shfl_xor(v.re, o, kWave);
      v.im += __shfl_xor(v.im, o, kWave);
    }
    return v;
  };
  for (int I = 0; I < bn; ++I) {
    if (I > 0) {
      const cplx<double>* Lb = F + (size_t)(2 * bn - 2 + I) * mm;
      cplx<double> acc = czero<double>();
      if (active)
        for (int c = l; c < bm; c += L) acc = cfma(Lb[r * bm + c], a[(I - 1) * bm + c], acc);
      acc = gsum(acc);
      if (active && l == 0) t[I * bm + r] = t[I * bm + r] - acc;
      lds_barrier();
    }
    const cplx<double>* G = F + (size_t)I * mm;
    cplx<double> acc = czero<double>();
    if (active)
      for (int c = l; c < bm; c += L) acc = cfma(G[r * bm + c], t[I * bm + c], acc);
    acc = gsum(acc);
    if (active && l == 0) a[I * bm + r] = acc;
    lds_barrier();
  }
  for (int I = bn - 2; I >= 0; --I) {
    const cplx<double>* H = F + (size_t)(bn + I) * mm;
    cplx<double> acc = czero<double>();
    if (active)
      for (int c = l; c < bm; c += L) acc = cfma(H[r * bm + c], a[(I + 1) * bm + c], acc);
    acc = gsum(acc);
    if (active && l == 0) a[I * bm + r] = a[I * bm + r] - acc;
    lds_barrier();
  }
}

}  // namespace detail

// y = E^{-1} t for one subdomain, workgroup-cooperative (NT threads).  `t` and `a`
// are d.ncp-entry LDS arrays (must not alias; entries from mx * my on are zero
// padding); the result overwrites `a` and `t` is used as scratch (its content is
// lost); `lc` holds the lower couplings staged by stage_lower (linear deflation).
// `fac` is the handle's factor base (the subdomain offset is applied here).  Block row
// r of each step is handled by a group of lanes that split its columns and reduce with
// DPP row operations, so every step costs one LDS-only barrier (two for the forward
// steps); factor entries are fetched a batch of steps at a time.
template <int NT>
__device__ __forceinline__ void coarse_solve(const SubDesc& d, const cplx<double>* __restrict__ fac,
                                             const cplx<double>* lc, cplx<double>* t, cplx<double>* a) {
  const cplx<double>* __restrict__ F = fac + d.goff;
  if (d.defl != 0) {
    detail::coarse_solve_paired<NT>(d, F, t, a);
    return;
  }
  const int L = coarse_group_lanes<NT>(d.mx);
  const int Q = (d.mx + L - 1) / L;
  // one ring shape per workgroup size (each instantiation costs registers in every
  // kernel that contains it): 512 threads cover mx <= 32 with 16 lanes per row, 256
  // threads with 8
  if constexpr (NT >= 512) {
    if (L == 16 && Q <= 2) detail::coarse_solve_ring<16, 2>(d, F, lc, t, a);
    else detail::coarse_solve_plain<NT>(d, F, lc, t, a);
  } else {
    if (L == 8 && Q <= 4) detail::coarse_solve_ring<8, 4>(d, F, lc, t, a);
    else detail::coarse_solve_plain<NT>(d, F, lc, t, a);
  }
}

}  // namespace ddh
