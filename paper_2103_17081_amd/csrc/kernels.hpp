// Host-side launchers of the ddhelm kernels (internal to the library).
#pragma once

#include "common.hpp"

namespace ddh {

// ---- set-up -----------------------------------------------------------------
hipError_t launch_assemble_coarse(const SubDesc* subs, int nsub, Consts cs, int local_bc, cplx<double>* Ec,
                                  hipStream_t st);
// Twisted block factorisation of E (linear deflation) or, through per-subdomain views, of
// the local matrices of the exact solves.  Both factorisations write, per subdomain j,
// pivmin[2 j] = the smallest |pivot| met and pivmin[2 j + 1] = the largest |entry| of the
// factored matrix (the scale set-up compares the pivots against).
hipError_t launch_factor_coarse_twisted(const SubDesc* subs, int nsub, const cplx<double>* Ec, cplx<double>* fac,
                                        double* pivmin, hipStream_t st);
hipError_t launch_factor_coarse_paired(const SubDesc* subs, int nsub, const cplx<double>* Ec, cplx<double>* fac,
                                       double* pivmin, hipStream_t st);

// ---- subdomain solves ---------------------------------------------------------
// Everything one batched launch of subdomain solves needs.  Packed fine vectors
// hold the tiles of all subdomains back to back (SubDesc::off), one copy per
// right-hand side (stride nfine).
template <typename T>
struct InnerArgs {
  const SubDesc* subs;
  const int* order;              // launch order of the solves (size nsub * nrhs), or null
  Consts cs;
  int local_bc;                  // 0 impedance, 1 Dirichlet
  const cplx<double>* fac;       // coarse block factors (twisted; paired rows for Bezier)
  const cplx<double>* Ec;        // coarse 9-point coefficients
  const cplx<double>* r;         // global right-hand sides [nrhs][ndof], or null: use F
  cplx<double>* z;               // global output [nrhs][ndof] (owned nodes), or null
  const cplx<double>* zadd;      // added to z at the owned nodes ([nrhs][ndof], stride ndof), or null
  cplx<T>* F;                    // packed local right-hand sides
  cplx<T>* U;                    // packed local solutions, or null
  const cplx<T>* guess;          // packed initial guesses, or null
  const float* gtile;            // guess tiles [nrhs * nsub][gT][gT][2] of the guess network, or null;
                                 // solve (rhs, sub) reads tile rhs * nsub + sub, values scaled by
                                 // sqrt(n_j) / ||f_j||
  int gT;
  cplx<T>* V;                    // Krylov bases: solve s at V + s_offset*(maxit+1)
  cplx<T>* W;                    // packed work vector
  cplx<T>* X;                    // packed work vector
  cplx<double>* R;               // per solve 2 maxit*maxit: the upper-triangular factor, then the
                                 // upper-triangular coordinates T of the Krylov candidates
  cplx<double>* Sc;              // per solve (maxit + 2) coarse vectors of max_nc: E^{-1} Z^T f, E^{-1} Z^T B x0,
                                 // E^{-1} Z^T B u~_i (kept so that the recovery needs no coarse solve), or null
  int* iters;                    // [nrhs][nsub] inner iterations, or null
  int* flags;                    // [nrhs][nsub] bit0 guess accepted, bit1 not converged
  const int* done;               // [nrhs] skip right-hand sides already converged, or null
  unsigned long long* counters;  // [5] total iterations, solves, max iterations, guesses accepted,
                                 //     algorithmic bytes
  long long nfine, ndof;
  long long rstride, zstride;    // per right-hand side strides of r and z (elements)
  const int* jdev;               // if set: r and z are advanced by (*jdev) * rslot / zslot
  long long rslot, zslot;        // (graph-captured outer steps read the step index on the device)
  int nrhs, maxit, max_nj, max_nc;
  double tol;
  int nt;                        // threads per workgroup: 256 or 512 (autotuned)
};

template <typename T>
hipError_t launch_inner_solve(const InnerArgs<T>& a, hipStream_t st);
// Raise the dynamic-LDS limit of the subdomain kernels once, at set-up (not while a
// stream is being captured).
template <typename T>
hipError_t configure_inner(int max_nj, int max_nc, int maxit);
template <typename T>
size_t inner_lds_bytes(int max_nj, int max_nc, int maxit);

// Kernel-level operations on packed vectors (one workgroup per subdomain).
template <typename T>
hipError_t launch_local_apply(const SubDesc* subs, int nsub, Consts cs, int local_bc, const cplx<T>* v,
                              cplx<T>* w, int max_nj, hipStream_t st);
template <typename T>
hipError_t launch_deflated_apply(const SubDesc* subs, int nsub, Consts cs, int local_bc,
                                 const cplx<double>* fac, const cplx<double>* Ec, const cplx<T>* v,
                                 cplx<T>* w, int max_nj, int max_nc, hipStream_t st);
hipError_t launch_restrict(const SubDesc* subs, int nsub, const cplx<double>* v, cplx<double>* t,
                           hipStream_t st);
hipError_t launch_prolong(const SubDesc* subs, int nsub, const cplx<double>* y, cplx<double>* v,
                          hipStream_t st);
hipError_t launch_coarse_solve(const SubDesc* subs, int nsub, const cplx<double>* fac,
                               const cplx<double>* Ec, const cplx<double>* t, cplx<double>* y, int max_nc,
                               hipStream_t st);
template <typename T>
hipError_t launch_gather(const SubDesc* subs, int nsub, Consts cs, const cplx<double>* r, cplx<T>* f,
                         long long nfine, long long ndof, int nrhs, hipStream_t st);
template <typename T>
hipError_t launch_scatter(const SubDesc* subs, int nsub, Consts cs, const cplx<T>* u, cplx<double>* z,
                          long long nfine, long long ndof, int nrhs, hipStream_t st);

// ---- plain multi-kernel subdomain solves (FP64, one right-hand side) -------------------
// The subdomain GMRES of the batched kernel as a sequence of batched launches per stage,
// iterated from the host (one synchronisation per inner iteration, no graph).
constexpr int kMultiMaxIt = 256;   // largest inner_maxit of this path
struct MultiArgs {
  const SubDesc* subs;
  Consts cs;
  int local_bc;
  const cplx<double>* fac;       // coarse block factors (twisted; paired rows for Bezier)
  const cplx<double>* Ec;        // coarse 9-point coefficients
  const cplx<double>* r;         // global right-hand side [ndof], or null: use F (unscaled, scaled in place)
  cplx<double>* z;               // global output (owned nodes), or null
  const cplx<double>* zadd;      // added to z at the owned nodes, or null
  const int* jdev;               // if set: r and z are advanced by (*jdev) * rslot / zslot
  long long rslot, zslot;
  const int* done;               // skip the solve when *done is set, or null
  cplx<double>* U;               // packed solutions (all tile nodes), or null
  // packed fine work vectors [nfine]
  cplx<double>* F;               // scaled local right-hand sides
  cplx<double>* W;               // deflated operator output / Arnoldi vector
  cplx<double>* T;               // stencil input
  cplx<double>* Bv;              // B v
  cplx<double>* X;               // x = V y
  cplx<double>* Zc;              // Z c of the recovery
  cplx<double>* V;               // Krylov bases: solve s at V + off_s (maxit + 1)
  // packed coarse vectors [ncoarse]
  cplx<double>* t;               // Z^T v
  cplx<double>* Yk;              // [maxit + 2][ncoarse]: slot 0 E^{-1} Z^T f, slot 2 + i E^{-1} Z^T B v_i
  cplx<double>* Cv;              // coarse vector of the recovery
  // per solve
  cplx<double>* H;               // Hessenberg column [nsub][maxit + 1]
  cplx<double>* g;               // rotated right-hand side [nsub][maxit + 1]
  double* csn;                   // rotation cosines [nsub][maxit]
  cplx<double>* snn;             // rotation sines [nsub][maxit]
  cplx<double>* R;               // upper-triangular factor [nsub][maxit][maxit] (column k at k maxit)
  double* fnorm;                 // ||R_j r||
  double* ref;                   // ||P f|| of the scaled problem
  double* wn;                    // ||P B v_k|| before orthogonalisation (breakdown scale)
  int* active;                   // 1 while the solve iterates
  int* notconv;                  // 1 when it stopped at maxit without converging
  int* nactive;                  // [1] active solves
  int* iters;                    // [nsub] inner iterations
  int* flags;                    // [nsub] bit1 not converged
  unsigned long long* counters;  // as InnerArgs
  long long nfine, ncoarse;
  int nsub, maxit, max_nj, max_nc;
  double tol;
};
// active_host: pinned host int the loop reads the active count into.
hipError_t run_multi_inner(const MultiArgs& a, int* active_host, hipStream_t st);

// ---- exact subdomain solves (FP64 twisted block factorisation of the local matrices) ---
struct DirectArgs {
  const SubDesc* subs;
  const int* order;              // launch order (size nsub * nrhs) or null
  Consts cs;
  int local_bc;
  const cplx<double>* ffac;      // twisted block factors of the local matrices
  const long long* foff;         // [nsub] factor offsets (complex<double> elements)
  const cplx<double>* r;         // global right-hand sides, or null: use F
  cplx<double>* z;               // global output (owned nodes), or null
  const cplx<double>* zadd;      // added to z at the owned nodes ([nrhs][ndof], stride ndof), or null
  const cplx<double>* F;         // packed right-hand sides [nrhs][nfine]
  cplx<double>* U;               // packed solutions, or null
  const int* done;
  int* iters;                    // [nrhs][nsub] set to 0, or null
  int* flags;                    // [nrhs][nsub] set to 0, or null
  unsigned long long* counters;  // [5] as InnerArgs: [1] solves, [4] algorithmic bytes
  long long nfine, ndof, rstride, zstride;
  const int* jdev;
  long long rslot, zslot;
  int nrhs, max_nj;
};
hipError_t launch_fine_coef(const SubDesc* subs, int nsub, Consts cs, int local_bc, cplx<double>* Bc,
                            hipStream_t st);
hipError_t launch_direct_solve(const DirectArgs& a, hipStream_t st);
size_t direct_lds_bytes(int max_nj);
hipError_t configure_direct(int max_nj);

// ---- static device scratch (the entry point that allocates nothing) -----------------
// Device address on the current device, and size, of the library's static scratch array
// (address looked up once per device with hipGetSymbolAddress).
hipError_t static_scratch(void** ptr, size_t* bytes);
// Zero `words` 8-byte words at p with a fill kernel (no memset node under graph capture).
hipError_t launch_zero_words(void* p, size_t words, hipStream_t st);

// ---- global FP64 operations (outer FGMRES) -----------------------------------------
hipError_t launch_global_apply(Consts cs, const cplx<double>* v, cplx<double>* w, int nrhs, hipStream_t st);

}  // namespace ddh
