// Device state and launchers of the outer FP64 FGMRES.
#pragma once

#include "common.hpp"

namespace ddh {

constexpr int kOuterMaxDots = 64;   // Gram-Schmidt coefficients per dot-product pass chunk

// The outer step index j of a kernel: read from device memory when `jdev` is set
// (kernels captured once into a graph and replayed for every step), else `jhost`.
struct StepRef {
  const int* jdev;
  int jhost;
  __device__ __forceinline__ int get() const { return jdev ? *jdev : jhost; }
};
inline StepRef host_step(int j) { return StepRef{nullptr, j}; }
inline StepRef device_step(const int* jdev) { return StepRef{jdev, 0}; }

// Per right-hand side: Hessenberg column, rotations, rotated rhs g, R factor (restart x
// restart, column-major), solution coefficients y, scalars.  All device pointers.
struct OuterState {
  cplx<double>* H;      // [nrhs][restart + 1] current column
  double* cs;           // [nrhs][restart]
  cplx<double>* sn;     // [nrhs][restart]
  cplx<double>* g;      // [nrhs][restart + 1]
  cplx<double>* R;      // [nrhs][restart][restart]
  cplx<double>* y;      // [nrhs][restart]
  cplx<double>* nrm2;   // norm-squared slot (read .re), stride nrm_stride
  int nrm_stride;
  double* res;          // [nrhs] residual estimate |g_{j+1}|
  double* hnext;        // [nrhs]
  double* atol;         // [nrhs] absolute tolerance rtol * ||f||
  int* steps;           // [nrhs] columns in the current cycle
  int* done;            // [nrhs]
  int* applies;         // [nrhs] preconditioner applications (step kernels entered with work)
  unsigned long long* sweep_bytes;   // [2] algorithmic bytes of the dot and update sweeps
  double rtol;
  int restart;
  int first_cycle;
};

hipError_t launch_global_apply_masked(Consts cs, const cplx<double>* v, long long vstride, cplx<double>* w,
                                      long long wstride, int nrhs, const int* done, hipStream_t st,
                                      StepRef sr = host_step(0), long long vslot = 0, long long wslot = 0);
hipError_t launch_advance_step(int* jdev, hipStream_t st);
hipError_t launch_residual(const cplx<double>* f, long long fstride, cplx<double>* w, long long wstride,
                           long long ndof, int nblk, int nrhs, hipStream_t st);
int outer_chunks(long long ndof);   // row chunks of the dots / update sweeps (part layout of launch_dots)
__host__ __device__ int dots2_chunks(long long ndof);   // row chunks of launch_dots2 (its part layout)
// segments of launch_reduce_chunks: part must hold nrhs * (dots2_chunks + dots2_segments) * pstride values
__host__ __device__ int dots2_segments(long long ndof);
hipError_t configure_outer();
hipError_t launch_fill_hash(cplx<double>* x, long long n, unsigned long long seed, hipStream_t st);   // dynamic-LDS limits of the bookkeeping kernels, at set-up
hipError_t launch_dots(const cplx<double>* basis, long long bstride, const cplx<double>* w, long long wstride,
                       long long ndof, int nvec, int with_norm, cplx<double>* part, int pstride, int nrhs,
                       const int* done, hipStream_t st);
// sums launch_dots' partials ([rhs][slot][chunk], nchunk = outer_chunks(ndof)) over the chunks
hipError_t launch_reduce_parts(const cplx<double>* part, int nchunk, int pstride, StepRef sr, int mul, int add,
                               int jmax, cplx<double>* out, int ostride, cplx<double>* H, int hstride, int mode,
                               int nrhs, const int* done, hipStream_t st);
hipError_t launch_update(const cplx<double>* basis, long long bstride, cplx<double>* w, long long wstride,
                         long long ndof, int nvec, const cplx<double>* coef, int cstride, double sign, int nrhs,
                         const int* done, hipStream_t st);
hipError_t launch_scale(const cplx<double>* w, long long wstride, cplx<double>* out, long long ostride,
                        long long ndof, const double* scale, int nblk, int nrhs, const int* done,
                        hipStream_t st);
// out[rhs][s] = sum over launch_dots2's chunks, s < mul * j + add (j from sr; jmax sizes the grid);
// the segment sums are kept in part after the chunk partials
hipError_t launch_reduce_chunks(const cplx<double>* part, long long ndof, int pstride, StepRef sr, int mul, int add,
                                int jmax, cplx<double>* out, int ostride, int nrhs, const int* done, hipStream_t st);
hipError_t launch_dots2(const cplx<double>* basis, long long bstride, const cplx<double>* x1, long long x1stride,
                        const cplx<double>* x2, long long x2stride, long long ndof, StepRef sr, int two, int jmax,
                        cplx<double>* part, int pstride, int nrhs, const int* done, hipStream_t st,
                        int max_blocks = 0);
hipError_t launch_dcgs2_step(const OuterState& s, StepRef sr, int jmax, long long ndof, const cplx<double>* dots,
                             int dstride, int has_w, cplx<double>* ca, cplx<double>* cb, int cstride,
                             cplx<double>* scal, int nrhs, hipStream_t st);
hipError_t launch_dcgs2_update(cplx<double>* basis, long long bstride, long long ndof, StepRef sr,
                               const cplx<double>* ca, const cplx<double>* cb, int cstride, const cplx<double>* scal,
                               int nrhs, const int* done, hipStream_t st);
hipError_t launch_backsolve(const OuterState& s, int nrhs, hipStream_t st);
hipError_t launch_cycle_init(const OuterState& s, int nrhs, hipStream_t st);

}  // namespace ddh
