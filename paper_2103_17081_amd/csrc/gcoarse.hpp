// Global coarse space of the two-level method: the step after the one-level
// preconditioner that the paper's conclusions name (Sec. 4), built on the same
// ingredients as the subdomain deflation of eq. 4, now for the global matrix A:
//
//   coarse grid lines at fine indices p_c = floor(c N / M + 1/2), c = 0..M;
//   Z_0 = Z^y kron Z^x, column c of the 1D factor the piecewise-linear hat of coarse
//         node c (1 at p_c, 0 at p_{c-1} and p_{c+1}), unknowns c = 1..M-1;
//   E_0 = Z_0^T A Z_0, a 9-point operator on the (M-1) x (M-1) coarse grid;
//   M^{-1} r = M_1^{-1} (r - A q) + q,  q = Z_0 E_0^{-1} Z_0^T r,
//
// with M_1^{-1} the one-level restricted Schwarz preconditioner of eq. 3.
//
// E_0 is block tridiagonal in the coarse rows (nb = M-1 blocks of n = M-1 unknowns).
// It is solved exactly in FP64 by block cyclic reduction: at every level the odd
// block rows of the remaining system are eliminated in terms of their even
// neighbours, which halves the system, until one block row remains.  With the
// inverse Binv_e of an eliminated row's diagonal block and its couplings A_e (lower)
// and C_e (upper),
//   P_e = -Binv_e A_e,  R_e = -Binv_e C_e,
//   Fm_i = -A_i Binv_{i-1},  Fp_i = -C_i Binv_{i+1}                (kept rows i)
//   B_i <- B_i + Fm_i C_{i-1} + Fp_i A_{i+1},  A_i <- Fm_i A_{i-1},  C_i <- Fp_i C_{i+1};
// the solve is then
//   reduction, level by level:   b_i += Fm_i b_{i-1} + Fp_i b_{i+1}
//   top:                         x_r = Binv_r b_r
//   back substitution, downward: x_e = Binv_e b_e + P_e x_{e-1} + R_e x_{e+1}
// (neighbours taken within the level).  On level 0 the couplings are the tridiagonal
// rows of E_0, so there the solve applies them directly and reads only Binv_e.  Every step of a level is a set of
// independent dense n x n matrix-vector products, spread over the whole chip, so the
// solve has 2 ceil(log2 nb) + 1 dependent launches instead of the 2 nb serial block
// steps of a block LU.  The set-up computes the dense blocks with a batched FP64
// GEMM and a batched Gauss-Jordan inverse with partial pivoting inside each block.
#pragma once

#include <vector>

#include "common.hpp"
#include "outer.hpp"

namespace ddh {

constexpr int kMaxGlobalCoarse = 1024;  // largest coarse block n = M - 1
constexpr int kBcrRhsGroup = 8;         // right-hand sides per pass of the solve kernel
constexpr int kBcrTile = 64;            // rows per tile of the factors' solve layout

// One dense block product of the solve: out = (base ? out : 0) + sum_t mat_t * in_t.
// Offsets are elements of the factor array (n x n matrices stored transposed, i.e.
// column-major) and of one right-hand side's coarse vector segment [b (nb n) | x (nb n)].
struct BcrTask {
  long long mat[3];
  int in[3];
  int out;
  int nt;
  int base;
  int pad;
};

// Set-up products: C = (acc ? C : 0) + sign * A B, n x n real row-major.  Operand
// arrays: 0 = the persistent factor, 1 = the set-up work blocks.
struct GemmTask {
  long long off[3];
  int arr[3];
  int acc;
  double sign;
};

// Inverse of a work block into the factor array (copy, then Gauss-Jordan in place).
struct InvTask {
  long long src, dst;
};

// Level-0 coupling update of the solve: out -= A_row in[0] + C_row in[1] (offsets in one
// right-hand side's coarse vector segment; has[s] = 0 drops a side).
struct SpTask {
  int out, row;
  int in[2];
  int has[2];
};

struct BcrPhase {
  int first, count;   // tasks [first, first + count) of the dense or sparse task table
  int kind;           // 0 dense block products (BcrTask), 1 level-0 couplings (SpTask)
};

class GlobalCoarse {
 public:
  int n_fine = 0;       // fine intervals N
  int M = 0;            // coarse intervals
  int nc = 0;           // coarse unknowns per direction, M - 1
  long long ncoarse = 0;
  long long ndof = 0;
  int nrhs = 1;
  long long nfac = 0;   // factor elements
  double min_pivot = 0.0;
  double max_entry = 0.0;        // largest |coefficient| of E_0 (scale of the pivot check)
  double kh2 = 0.0;
  // device
  int* pos = nullptr;            // [M + 1] coarse grid lines
  int* cell = nullptr;           // [N + 1] coarse interval containing each fine index
  double* E0c = nullptr;         // [ncoarse][9] coefficients, neighbour (dx, dy) at 3 (dy + 1) + (dx + 1)
  double* emax_d = nullptr;      // per-workgroup largest |coefficient| of E_0
  double* fac = nullptr;         // block cyclic reduction factors (real: A and Z_0 are real)
  BcrTask* tasks = nullptr;
  SpTask* sptasks = nullptr;
  cplx<double>* cv = nullptr;    // [nrhs][2 ncoarse] coarse vectors b | x
  cplx<double>* q = nullptr;     // [nrhs][ndof] coarse correction Z_0 x
  cplx<double>* w = nullptr;     // [nrhs][ndof] corrected residual r - A q
  std::vector<BcrPhase> phases;  // solve launches in order
  std::vector<void*> allocs;

  ~GlobalCoarse();
  // Build Z_0, E_0 and its factors on the device (synchronises st).  Returns a HIP
  // error; a non-finite or zero pivot leaves min_pivot <= 0.
  hipError_t setup(int n, int m, double k, int nrhs, hipStream_t st);
  // The first nr right-hand sides (nr <= nrhs); those with done set are skipped.
  // b = Z_0^T r into the b segments (r: rhs stride rstride, advanced by jdev * rslot).
  hipError_t restrict_rhs(const cplx<double>* r, long long rstride, const int* jdev, long long rslot,
                          const int* done, int nr, hipStream_t st);
  // x = E_0^{-1} b (block cyclic reduction).
  hipError_t solve(int nr, hipStream_t st);
  // q = Z_0 x and w = r - A q.
  hipError_t correct(const cplx<double>* r, long long rstride, const int* jdev, long long rslot, const int* done,
                     int nr, hipStream_t st);
  // Factor bytes one solve reads (the algorithmic traffic of the coarse solve).
  long long solve_bytes() const { return solve_bytes_; }

 private:
  long long solve_bytes_ = 0;
  template <typename T>
  hipError_t alloc(T** p, size_t count);
};

}  // namespace ddh
