// Coarse deflation operator E = Z^T B Z (Sec. 2, eq. 4) for linear interpolation
// Z = Z^y kron Z^x (eq. 5), and its FP64 block factorisations.
//
// With coarse nodes ordered x fastest, E couples a coarse node only to its 3 x 3
// coarse neighbours, so E is block tridiagonal in the coarse rows: diagonal blocks
// D_i, sub-diagonal L_i (row i to row i-1), super-diagonal U_i (row i to row i+1),
// each an mx x mx tridiagonal matrix.  E is complex symmetric (B is), so U_i = L_{i+1}^T;
// the factorisation and the solve both take U_i from the stored L_{i+1}, which keeps the
// factored matrix exactly symmetric whatever the rounding of the assembly.
//
// Twisted block factorisation (elimination from both ends towards the middle row
// p = (my - 1) / 2), without block pivoting:
//   top,    i < p:  G_i = (D_i - L_i H_{i-1})^{-1},   H_i = G_i U_i;
//   bottom, i > p:  K_i = (D_i - U_i J_{i+1})^{-1},   J_i = K_i L_i;
//   middle:         M   = (D_p - L_p H_{p-1} - U_p J_{p+1})^{-1}.
// Solve E y = t:
//   a_i = G_i (t_i - L_i a_{i-1}) for i < p  and  b_i = K_i (t_i - U_i b_{i+1}) for i > p,
//   both sweeps side by side;  y_p = M (t_p - L_p a_{p-1} - U_p b_{p+1});
//   y_i = a_i - H_i y_{i+1} (i < p)  and  y_i = b_i - J_i y_{i-1} (i > p), side by side.
// That is my sequential dense mx x mx products (against 2 my - 1 for the one-ended block
// LU), with the same 2 my - 1 stored blocks and the same bytes streamed.  Each inverse
// is formed by Gauss-Jordan elimination with partial pivoting.
//
// Storage per subdomain at SubDesc::goff (complex<double>), mx*mx row-major blocks
// (element (r, c) at r*mx + c): G_0..G_{p-1}, H_0..H_{p-1}, K_{p+1}..K_{my-1},
// J_{p+1}..J_{my-1}, M.  E itself is kept as nine coefficients per coarse node, offset
// index o = 3*(dy+1) + (dx+1) for the neighbour (cx+dx, cy+dy).
//
// The exact local solves factor the local matrices B_j the same way (block size nx, ny
// block rows), through the same set-up kernel and solve.
#pragma once

#include "common.hpp"

namespace ddh {

constexpr int kMaxMx = 128;   // largest coarse block (mx) the kernels support

__host__ __device__ __forceinline__ long long coarse_factor_size(int mx, int my) {
  return (long long)(2 * my - 1) * mx * mx;
}

// Twisted factorisation: middle row and block offsets (in units of mx*mx blocks).
__host__ __device__ __forceinline__ int twist_row(int my) { return (my - 1) / 2; }
__host__ __device__ __forceinline__ int tw_G(int i) { return i; }
__host__ __device__ __forceinline__ int tw_H(int p, int i) { return p + i; }
__host__ __device__ __forceinline__ int tw_K(int p, int i) { return p + i - 1; }
__host__ __device__ __forceinline__ int tw_J(int my, int i) { return my + i - 2; }
__host__ __device__ __forceinline__ int tw_M(int my) { return 2 * my - 2; }

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

// ---- twisted solve of E (linear deflation; layout above) ----------------------------
// The workgroup is split into two halves of Half threads: half 0 runs the top sweep
// (and the middle row), half 1 the bottom sweep.  Step s of the solve:
//   s < nf = my - 1 - p:  a_s (top, if s < p) and b_{my-1-s} (bottom);
//   s = nf:               the coupled middle right-hand side, then y_p;
//   s > nf:               y_{p-1-(s-nf-1)} (top) and y_{p+1+(s-nf-1)} (bottom).
// a, b and y share the LDS array `a` (row i at a + i mx); t is used as scratch.
// lower(i, c, e): coupling of unknown c of row i to unknown c+e-1 of row i-1 (for E, the
// staged lc[3 (i mx + c) + e]); the upper coupling of unknown c of row i-1 to c+e-1 of
// row i is lower(i, c+e-1, 2-e).

// Factor block (mx*mx units) half h reads at step s, or -1.
__device__ __forceinline__ int tw_step_block(int h, int s, int p, int my) {
  const int nf = my - 1 - p;
  if (s < nf) return h == 0 ? (s < p ? tw_G(s) : -1) : tw_K(p, my - 1 - s);
  if (s == nf) return h == 0 ? tw_M(my) : -1;
  const int b = s - nf - 1;
  if (h == 0) return p - 1 - b >= 0 ? tw_H(p, p - 1 - b) : -1;
  return p + 1 + b <= my - 1 ? tw_J(my, p + 1 + b) : -1;
}

// `v` if `keep`, else 0 (a select, not a branch).
__device__ __forceinline__ cplx<double> keep_c(bool keep, cplx<double> v) {
  return cplx<double>{keep ? v.re : 0.0, keep ? v.im : 0.0};
}

// t_{i+1} -= L_{i+1} a_i (top) for unknown c.  Neighbours outside the row are read at c
// with a zero coupling, so all operands are loaded without branches (same sum).
template <typename Lower>
__device__ __forceinline__ void tw_couple_down(int mx, Lower lower, int i, int c, cplx<double>* t,
                                               const cplx<double>* a) {
  const cplx<double>* ap = a + i * mx + c;
  const bool lo = c > 0, hi = c < mx - 1;
  const cplx<double> l0 = keep_c(lo, lower(i + 1, c, 0)), l2 = keep_c(hi, lower(i + 1, c, 2));
  const cplx<double> am = ap[lo ? -1 : 0], a0 = ap[0], ap1 = ap[hi ? 1 : 0];
  cplx<double> v = t[(i + 1) * mx + c] - lower(i + 1, c, 1) * a0;
  v = v - l0 * am;
  v = v - l2 * ap1;
  t[(i + 1) * mx + c] = v;
}

// t_{i-1} -= U_{i-1} b_i (bottom) for unknown c, U_{i-1} read as L_i^T.
template <typename Lower>
__device__ __forceinline__ void tw_couple_up(int mx, Lower lower, int i, int c, cplx<double>* t,
                                             const cplx<double>* a) {
  const cplx<double>* bp = a + i * mx + c;
  const bool lo = c > 0, hi = c < mx - 1;
  const cplx<double> u0 = keep_c(lo, lower(i, lo ? c - 1 : c, 2)), u2 = keep_c(hi, lower(i, hi ? c + 1 : c, 0));
  const cplx<double> bm = bp[lo ? -1 : 0], b0 = bp[0], bp1 = bp[hi ? 1 : 0];
  cplx<double> v = t[(i - 1) * mx + c] - lower(i, c, 1) * b0;
  v = v - u0 * bm;
  v = v - u2 * bp1;
  t[(i - 1) * mx + c] = v;
}

// t_p -= L_p a_{p-1} + U_p b_{p+1} for unknown c.
template <typename Lower>
__device__ __forceinline__ void tw_couple_middle(int mx, int my, int p, Lower lower, int c, cplx<double>* t,
                                                 const cplx<double>* a) {
  if (p > 0) tw_couple_down(mx, lower, p - 1, c, t, a);
  if (p < my - 1) tw_couple_up(mx, lower, p + 1, c, t, a);
}

// Factor blocks of Depth consecutive steps are loaded together into registers (clamped
// indices, straight-line code) before those steps run.  Lane l of row group r of a half
// owns columns l + q L, q < Q (mx <= L Q, rows Half / L >= mx).
template <int L, int Q, int Depth, int Half, typename Lower>
__device__ __forceinline__ void twisted_solve_ring(int mx, int my, const cplx<double>* __restrict__ F, Lower lower,
                                                   cplx<double>* t, cplx<double>* a) {
  const int mm = mx * mx, p = twist_row(my), nf = my - 1 - p, nsteps = 2 * nf + 1;
  const int h = threadIdx.x / Half, ht = threadIdx.x % Half;
  const int r = ht / L, l = ht % L;
  const bool active = r < mx;
  // Columns a lane does not own read column 0 with a zero factor entry, so every step
  // reads its operands without branches (adding 0 * x leaves the sum unchanged).
  int col[Q], eoff[Q];
  bool ok[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    ok[q] = active && l + q * L < mx;
    col[q] = ok[q] ? l + q * L : 0;
    eoff[q] = ok[q] ? r * mx + col[q] : 0;
  }
  cplx<double> ring[Depth][Q];
  for (int s0 = 0; s0 < nsteps; s0 += Depth) {
#pragma unroll
    for (int u = 0; u < Depth; ++u) {
      const int blk = max(tw_step_block(h, s0 + u, p, my), 0);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const cplx<double> fv = F[(size_t)blk * mm + eoff[q]];
        ring[u][q].re = ok[q] ? fv.re : 0.0;
        ring[u][q].im = ok[q] ? fv.im : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < Depth; ++u) {
      const int s = s0 + u;
      if (s >= nsteps) break;
      if (s < nf) {
        // a_s = G_s t_s (top, s < p), b_i = K_i t_i (bottom, i = my-1-s)
        const int i = h == 0 ? s : my - 1 - s;
        const bool on = h == 1 || s < p;
        cplx<double> acc = czero<double>();
        if (on) {
#pragma unroll
          for (int q = 0; q < Q; ++q) acc = cfma(ring[u][q], t[i * mx + col[q]], acc);
        }
        acc.re = row_sum<L>(acc.re);
        acc.im = row_sum<L>(acc.im);
        if (on && active && l == 0) a[i * mx + r] = acc;
        lds_barrier();
        if (ht < mx) {
          if (h == 0) {
            if (s + 1 < p) tw_couple_down(mx, lower, s, ht, t, a);
          } else {
            if (i - 1 > p) tw_couple_up(mx, lower, i, ht, t, a);
          }
        }
        lds_barrier();
      } else if (s == nf) {
        if (h == 0 && ht < mx) tw_couple_middle(mx, my, p, lower, ht, t, a);
        lds_barrier();
        cplx<double> acc = czero<double>();
        if (h == 0) {
#pragma unroll
          for (int q = 0; q < Q; ++q) acc = cfma(ring[u][q], t[p * mx + col[q]], acc);
        }
        acc.re = row_sum<L>(acc.re);
        acc.im = row_sum<L>(acc.im);
        if (h == 0 && active && l == 0) a[p * mx + r] = acc;
        lds_barrier();
      } else {
        // y_i = a_i - H_i y_{i+1} (top), y_i = b_i - J_i y_{i-1} (bottom); a_i is read
        // before the product so that its load overlaps it
        const int b = s - nf - 1;
        const int i = h == 0 ? p - 1 - b : p + 1 + b;
        const bool on = h == 0 ? i >= 0 : i <= my - 1;
        const int src = h == 0 ? i + 1 : i - 1;
        const cplx<double> ai = a[(on ? i : p) * mx + (active ? r : 0)];
        cplx<double> acc = czero<double>();
        if (on) {
#pragma unroll
          for (int q = 0; q < Q; ++q) acc = cfma(ring[u][q], a[src * mx + col[q]], acc);
        }
        acc.re = row_sum<L>(acc.re);
        acc.im = row_sum<L>(acc.im);
        if (on && active && l == 0) a[i * mx + r] = ai - acc;
        lds_barrier();
      }
    }
  }
}

// Same steps for any mx <= kMaxMx: factor entries read as they are used, shuffle
// reductions over groups of L = coarse_group_lanes<Half>(mx) lanes.
template <int Half, typename Lower>
__device__ __forceinline__ void twisted_solve_plain(int mx, int my, const cplx<double>* __restrict__ F, Lower lower,
                                                    cplx<double>* t, cplx<double>* a) {
  const int mm = mx * mx, p = twist_row(my), nf = my - 1 - p, nsteps = 2 * nf + 1;
  const int L = coarse_group_lanes<Half>(mx);
  const int h = threadIdx.x / Half, ht = threadIdx.x % Half;
  const int r = ht / L, l = ht % L;
  const bool active = r < mx;
  auto gsum = [&](cplx<double> v) {
    for (int o = L >> 1; o > 0; o >>= 1) {
      v.re += __shfl_xor(v.re, o, kWave);
      v.im += __shfl_xor(v.im, o, kWave);
    }
    return v;
  };
  auto product = [&](int blk, const cplx<double>* x) {
    cplx<double> acc = czero<double>();
    if (active)
      for (int c = l; c < mx; c += L) acc = cfma(F[(size_t)blk * mm + r * mx + c], x[c], acc);
    return gsum(acc);
  };
  for (int s = 0; s < nsteps; ++s) {
    const int blk = tw_step_block(h, s, p, my);
    if (s < nf) {
      const int i = h == 0 ? s : my - 1 - s;
      const cplx<double> acc = product(max(blk, 0), t + i * mx);
      if (blk >= 0 && active && l == 0) a[i * mx + r] = acc;
      lds_barrier();
      if (ht < mx) {
        if (h == 0) {
          if (s + 1 < p) tw_couple_down(mx, lower, s, ht, t, a);
        } else {
          if (i - 1 > p) tw_couple_up(mx, lower, i, ht, t, a);
        }
      }
      lds_barrier();
    } else if (s == nf) {
      if (h == 0 && ht < mx) tw_couple_middle(mx, my, p, lower, ht, t, a);
      lds_barrier();
      const cplx<double> acc = product(tw_M(my), t + p * mx);
      if (h == 0 && active && l == 0) a[p * mx + r] = acc;
      lds_barrier();
    } else {
      const int b = s - nf - 1;
      const int i = h == 0 ? p - 1 - b : p + 1 + b;
      const int src = h == 0 ? i + 1 : i - 1;
      const cplx<double> acc = blk >= 0 ? product(blk, a + src * mx) : czero<double>();
      if (blk >= 0 && active && l == 0) a[i * mx + r] = a[i * mx + r] - acc;
      lds_barrier();
    }
  }
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
  // the two halves run the two sweeps: 512 threads give 8 lanes per block row (mx <= 32),
  // 256 threads 4 lanes; rings of 3 steps (a deeper ring makes the subdomain-solve kernel
  // spill the ring's column offsets to scratch inside the step loop, where each reload
  // waits for every factor load in flight)
  auto lower = [lc, mx = d.mx](int i, int c, int e) { return lc[3 * (i * mx + c) + e]; };
  if (d.mx <= 32) {
    if constexpr (NT >= 512) detail::twisted_solve_ring<8, 4, 3, NT / 2>(d.mx, d.my, F, lower, t, a);
    else detail::twisted_solve_ring<4, 8, 3, NT / 2>(d.mx, d.my, F, lower, t, a);
  } else {
    detail::twisted_solve_plain<NT / 2>(d.mx, d.my, F, lower, t, a);
  }
}

}  // namespace ddh
