// Exact subdomain solves with an FP64 block factorisation of each local matrix: the direct-solve
// baseline against which the paper measures its inexact solves (Sec. 3, Table 1).
//
// With the tile's nodes ordered x fastest, the local P1 matrix B_j is block tridiagonal
// in the rows of the tile: diagonal blocks couple a row to itself (W, C, E), the lower
// block a row to the row below (S and SW for the SW->NE cell diagonal), the upper block
// to the row above (N, NE).  B_j is complex symmetric, and the same twisted block
// factorisation as the coarse deflation matrices (coarse.hpp: elimination from both ends
// towards the middle row, upper couplings read as the transposed lower ones) is built at
// set-up, once per subdomain; every solve is ny sequential dense nx x nx products, the
// two sweeps side by side.  One workgroup per (subdomain, right-hand side): gather R_j r,
// the block sweeps with the lower couplings taken from the stencil's row classes, scatter
// of the owned nodes.
#include "coarse.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace ddh {

// Bc[(off + n) * 9 + o] = coupling of local node n to its neighbour (dx, dy),
// o = 3 (dy + 1) + (dx + 1): the local matrix in the 9-coefficient layout of E.
__global__ void __launch_bounds__(kBlock) fine_coef_kernel(const SubDesc* __restrict__ subs, Consts cs,
                                                            int local_bc, cplx<double>* __restrict__ Bc) {
  const SubDesc d = subs[blockIdx.x];
  __shared__ cplx<double> tab[kClasses * kStencilPts];
  build_class_table<double>(d.robin, cs.kh, cs.kh2, tab);
  __syncthreads();
  const int nj = d.nx * d.ny;
  // stencil point -> 9-coefficient slot
  const int slot[kStencilPts] = {4, 3, 5, 1, 7, 0, 8};
  for (int e = threadIdx.x; e < nj * 9; e += blockDim.x) {
    const int n = e / 9, o = e % 9;
    const int lj = n / d.nx, li = n - lj * d.nx;
    const int dx = o % 3 - 1, dy = o / 3 - 1;
    cplx<double> v = czero<double>();
    if (li + dx >= 0 && li + dx < d.nx && lj + dy >= 0 && lj + dy < d.ny) {
      const int cls = local_bc == 0 ? node_class(d.i0 + li, d.j0 + lj, d.ax, d.bx, d.ay, d.by) : 4;
      for (int s = 0; s < kStencilPts; ++s)
        if (slot[s] == o) v = tab[cls * kStencilPts + s];
    }
    Bc[(d.off + n) * 9 + o] = v;
  }
}

hipError_t launch_fine_coef(const SubDesc* subs, int nsub, Consts cs, int local_bc, cplx<double>* Bc,
                            hipStream_t st) {
  hipLaunchKernelGGL(fine_coef_kernel, dim3(nsub), dim3(kBlock), 0, st, subs, cs, local_bc, Bc);
  return hipGetLastError();
}

size_t direct_lds_bytes(int max_nj) {
  return 64 * sizeof(cplx<double>) + 2 * (size_t)max_nj * sizeof(cplx<double>);
}

template <int NT>
__global__ void __launch_bounds__(NT) direct_solve_kernel(DirectArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int sidx = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
  const int nsub = a.cs.nsub;
  const int rhs = sidx / nsub, sub = sidx - rhs * nsub;
  if (a.done && a.done[rhs]) return;
  const SubDesc d = a.subs[sub];
  cplx<double>* tab = (cplx<double>*)smem;
  cplx<double>* t = tab + 64;
  cplx<double>* x = t + a.max_nj;
  const int tid = threadIdx.x, nx = d.nx, ny = d.ny, nj = nx * ny, ldg = a.cs.n - 1;
  build_class_table<double>(d.robin, a.cs.kh, a.cs.kh2, tab);
  const long long jstep = a.jdev ? (long long)*a.jdev : 0;
  const cplx<double>* __restrict__ rin = a.r ? a.r + jstep * a.rslot + (long long)rhs * a.rstride : nullptr;
  cplx<double>* __restrict__ zout = a.z ? a.z + jstep * a.zslot + (long long)rhs * a.zstride : nullptr;
  for (int n = tid; n < nj; n += NT) {
    const int lj = n / nx, li = n - lj * nx;
    t[n] = rin ? rin[(long long)(d.j0 + lj - 1) * ldg + (d.i0 + li - 1)] : a.F[(long long)rhs * a.nfine + d.off + n];
  }
  __syncthreads();
  // coupling of node (c, i) to (c + e - 1, i - 1): SW, S, and no SE for the SW->NE diagonal
  const int lbc = a.local_bc;
  auto lower = [&](int i, int c, int e) -> cplx<double> {
    if (e == 2) return czero<double>();
    const int cls = lbc == 0 ? node_class(d.i0 + c, d.j0 + i, d.ax, d.bx, d.ay, d.by) : 4;
    return tab[cls * kStencilPts + (e == 0 ? kSW : kS)];
  };
  const cplx<double>* __restrict__ F = a.ffac + a.foff[sub];
  // the two halves of the workgroup run the two sweeps of the twisted factorisation; for
  // 33..64-wide tiles the factor entries of one step are loaded at a time (179 us per
  // application on the large workload, against 189 and 193 us with 2 and 3 steps ahead)
  if (nx <= 32) detail::twisted_solve_ring<8, 4, 8, NT / 2>(nx, ny, F, lower, t, x);
  else if (nx <= 64) detail::twisted_solve_ring<4, 16, 1, NT / 2>(nx, ny, F, lower, t, x);
  else detail::twisted_solve_plain<NT / 2>(nx, ny, F, lower, t, x);
  for (int n = tid; n < nj; n += NT) {
    if (a.U) a.U[(long long)rhs * a.nfine + d.off + n] = x[n];
    if (zout) {
      const int lj = n / nx, li = n - lj * nx;
      const int gi = d.i0 + li, gj = d.j0 + lj;
      if (gi >= d.oi0 && gi <= d.oi1 && gj >= d.oj0 && gj <= d.oj1) {
        const long long gidx = (long long)(gj - 1) * ldg + (gi - 1);
        zout[gidx] = a.zadd ? x[n] + a.zadd[(long long)rhs * a.ndof + gidx] : x[n];
      }
    }
  }
  if (tid == 0) {
    if (a.iters) a.iters[sidx] = 0;
    if (a.flags) a.flags[sidx] = 0;
  }
  if (tid == 0 && a.counters) {
    atomicAdd(a.counters + 1, 1ull);
    const unsigned long long own = (unsigned long long)(d.oi1 - d.oi0 + 1) * (d.oj1 - d.oj0 + 1);
    const unsigned long long bytes =
        16ull * (unsigned long long)coarse_factor_size(nx, ny) + 16ull * nj + (a.zadd ? 32ull : 16ull) * own;
    atomicAdd(a.counters + 4, bytes);
  }
}

hipError_t launch_direct_solve(const DirectArgs& a, hipStream_t st) {
  const int nblocks = a.cs.nsub * a.nrhs;
  hipLaunchKernelGGL(direct_solve_kernel<kInnerThreads>, dim3(nblocks), dim3(kInnerThreads),
                     direct_lds_bytes(a.max_nj), st, a);
  return hipGetLastError();
}

hipError_t configure_direct(int max_nj) {
  return hipFuncSetAttribute((const void*)direct_solve_kernel<kInnerThreads>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)direct_lds_bytes(max_nj));
}

}  // namespace ddh
