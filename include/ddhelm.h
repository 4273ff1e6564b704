/*
 * ddhelm -- MI355X (gfx950) solver for the P1-discretised 2D Dirichlet Helmholtz
 * problem  -Delta u - k^2 u = f  on (0,1)^2,  u = 0 on the boundary
 * (Bootland, Dwarka, Jolivet, Dolean, Vuik, arXiv:2103.17081, Sec. 2, eqs. 1-2),
 * by outer FGMRES (Sec. 3) preconditioned with one-level restricted additive
 * Schwarz (Sec. 2, eq. 3) whose subdomain systems are solved inexactly by GMRES
 * preconditioned with two-level deflation (Sec. 2, eqs. 4-5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: N intervals per edge, h = 1/N; the unknowns are the (N-1)^2 interior nodes
 *   (i, j), 1 <= i, j <= N-1, stored x fastest: index (j-1)(N-1) + (i-1)
 *   (the ordering Sec. 2 assumes for the Kronecker deflation matrix, eq. 5).
 * Global vectors: interleaved complex128 (re, im), [nrhs][ndof], device memory,
 *   contiguous, owned by the caller.
 * Packed subdomain vectors: the tiles of all subdomains back to back, tile j at
 *   dd_layout's fine offset, nx*ny nodes x fastest; complex128 or complex64 as the
 *   entry point states; [nrhs][nfine] where an entry point says so.
 * Packed coarse vectors: complex128, subdomain j at its coarse offset, mx*my values.
 * Streams: `stream` is a hipStream_t (NULL = the default stream); all device work
 *   is enqueued on it.  Entry points that return host values synchronise it.
 * Ownership: the handle owns all internal device memory (allocated by dd_setup,
 *   freed by dd_destroy); dd_apply_preconditioner and dd_solve allocate nothing.
 * Errors: every entry point returns a dd_status; on failure dd_last_error() gives
 *   a message (thread-local).  Arguments are validated before any device work.
 * Threads: a handle may be used by one host thread at a time.
 */
#ifndef DDHELM_H
#define DDHELM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd_handle dd_handle;

typedef enum {
  DD_OK = 0,
  DD_EINVAL = 1,      /* invalid argument or unsupported configuration */
  DD_ENOMEM = 2,      /* device allocation failed */
  DD_EHIP = 3,        /* HIP runtime error */
  DD_ESINGULAR = 4,   /* a factored matrix (a coarse E_j, a local B_j of the exact solves, the global
                         coarse E_0) is singular to working precision: a zero or non-finite pivot,
                         or min |pivot| < 1e-12 max |entry| (k^2 at an eigenvalue of a local or
                         coarse pencil); the message gives the ratio */
  DD_ENOTCONV = 5,    /* outer FGMRES hit outer_maxit; the best iterate is still written */
  DD_EWEIGHTS = 6     /* dd_net_load: the weights file is missing, malformed, inconsistent with its
                         widths, or holds a non-finite parameter */
} dd_status;

enum { DD_LOCAL_IMPEDANCE = 0, DD_LOCAL_DIRICHLET = 1 };
enum { DD_DEFLATION_LINEAR = 0, DD_DEFLATION_BEZIER = 1 };
enum { DD_LOCAL_DEFLATED_GMRES = 0, DD_LOCAL_DIRECT = 1 };
enum { DD_INNER_FUSED = 0, DD_INNER_MULTI = 1 };

/* Problem and solver parameters.  Start from dd_default_params(). */
typedef struct {
  double k;            /* wave number (Sec. 2, eq. 1) */
  double ppwl;         /* points per wavelength; used when n_intervals <= 0:
                          N = ceil(k * ppwl / (2 pi)), so h <= 2 pi / (k ppwl) (Sec. 2) */
  int n_intervals;     /* N > 0 overrides ppwl */
  int px, py;          /* subdomains per direction (Cartesian partition, Sec. 2) */
  const int* cuts_x;   /* optional host array of px+1 cut points 0 = c_0 < ... < c_px = N;
                          NULL = uniform c_p = floor(p N / px).  Copied by dd_setup. */
  const int* cuts_y;   /* same for y */
  int overlap;         /* mesh-element layers appended on each interior side (>= 1; Sec. 3) */
  int local_bc;        /* DD_LOCAL_IMPEDANCE: B_j = K_j - k^2 M_j - i k M_Gamma_j (optimised
                          interface condition); DD_LOCAL_DIRICHLET: A_j = R_j A R_j^T (eq. 3) */
  int deflation;       /* DD_DEFLATION_LINEAR (H = 2h interpolation) or DD_DEFLATION_BEZIER (the
                          quadratic rational Bezier stencil 1/8 [1 4 6 4 1] of Sec. 2, read as Z^T) */
  int inner_precision; /* 64: complex128 subdomain Krylov work; 32: complex64.  The coarse
                          solve and the outer FGMRES are FP64 in both. */
  double inner_tol;    /* relative tolerance of each subdomain GMRES on ||P_j f_j|| (Sec. 3) */
  int inner_maxit;     /* subdomain GMRES iterations (no restart) */
  double outer_tol;    /* FGMRES relative residual tolerance (Sec. 3: 1e-6) */
  int outer_maxit;     /* total FGMRES iterations */
  int outer_restart;   /* FGMRES restart length; <= 0 means outer_maxit (no restart) */
  int nrhs;            /* independent right-hand sides solved together */
  int use_graph;       /* 1: outer steps replayed from a captured hipGraph (default), 0: launched one by one */
  int graph_steps;     /* outer steps per graph replay; convergence is read back once per replay */
  int local_solver;    /* DD_LOCAL_DEFLATED_GMRES (default): inexact deflated-GMRES subdomain solves;
                          DD_LOCAL_DIRECT: exact solves with the FP64 twisted block
                          factorisation of each local matrix (the direct-solve baseline of
                          Sec. 3, Table 1); needs inner_precision 64,
                          ignores the inner tolerances and the deflation choice */
  int coarse_intervals; /* 0 (default): the one-level preconditioner of eq. 3.  M >= 2: two-level
                          method with a global coarse space, the extension the paper's
                          conclusions propose (Sec. 4): coarse grid lines at fine indices
                          p_c = floor(c N / M + 1/2), c = 0..M; Z_0 = Z^y kron Z^x with the
                          piecewise-linear hats of the interior lines (the global analogue of the
                          linear deflation of eq. 5); E_0 = Z_0^T A Z_0 factored exactly (FP64
                          block cyclic reduction); each application is
                          M^{-1} r = M_1^{-1} (r - A Q_0 r) + Q_0 r, Q_0 = Z_0 E_0^{-1} Z_0^T, with
                          M_1^{-1} the one-level preconditioner.  Needs M <= N and M - 1 <= 1024. */
  int inner_launch;    /* DD_INNER_FUSED (default): every subdomain solve of a preconditioner
                          application runs inside one batched launch (one workgroup per solve, the
                          whole GMRES iteration in the kernel).  DD_INNER_MULTI: the plain form of
                          the same deflated GMRES -- one batched launch per stage (stencil,
                          restriction, coarse solve, prolongation, Gram-Schmidt pass, rotation)
                          with the iteration loop on the host and one host synchronisation per
                          inner iteration; needs inner_precision 64, nrhs 1, use_graph 0,
                          inner_maxit <= 256 and no guess network. */
} dd_params;

typedef struct {
  int outer_iters;             /* FGMRES columns (Krylov dimension) used, summed over restart
                                  cycles: the count of preconditioned directions the solution needed */
  int precond_applies;         /* preconditioner applications performed; the delayed
                                  reorthogonalisation decides convergence one step late, so this is
                                  outer_iters + 1 per cycle when the solve converges */
  int converged;               /* all right-hand sides reached outer_tol */
  long long inner_iters_total; /* GMRES iterations over all subdomain solves */
  long long subdomain_solves;  /* subdomain solves performed */
  int inner_iters_max;
  long long guesses_accepted;
  double final_res_estimate;   /* max over rhs of the FGMRES estimate / ||f|| */
  /* Phase timings from HIP events recorded on `stream` around each launch group
     (milliseconds, summed over the solve), and launch counts. */
  double ms_inner;             /* batched subdomain-solve kernel (preconditioner) */
  double ms_spmv;              /* global stencil A z_j */
  double ms_orth;              /* outer delayed CGS2: dot sweep + bookkeeping + update sweep */
  double ms_other;             /* of which the bookkeeping (reductions, Givens rotations) */
  int inner_launches;          /* outer steps enqueued (including no-op steps after convergence
                                  inside a graph replay) */
  /* Algorithmic bytes of the subdomain-solve kernel summed over its launches: per solve,
     gather 16 n_j + scatter 16 owned_j (32 when the two-level correction is added) +
     (k_j + 1) coarse-factor reads of 16 ((2 my - 1) mx^2 + 3 mx my) bytes + the coarse vectors kept for the
     recovery 16 nc (2 k_j + 2) + Krylov traffic s n_j (1 + 3 k_j + 3 k_j (k_j + 1) / 2) when
     k_j > 0 (basis writes 1 + 2 k_j, three delayed-CGS2 sweeps per iteration reading
     3 k_j (k_j + 1) / 2 basis vectors in all, final combination k_j) + local rhs write/read
     2 s n_j, with s = 8 (FP32) or 16 bytes per complex value. */
  double inner_bytes;
  /* The two basis sweeps of the outer delayed CGS2 (events around each launch):
     dot sweep reads the j basis vectors and two vectors, 16 nd (j + 2) bytes at step j;
     update sweep reads the j basis vectors and two vectors and writes two,
     16 nd (j + 4) bytes (nd unknowns, complex128). */
  double ms_dots, ms_update;
  double dots_bytes, update_bytes;
  int graph_replays;           /* graph launches (0 when use_graph is off) */
  int timed_steps;             /* outer steps launched one by one; the per-phase times above cover
                                  only these (events cannot be timed inside graph replays) */
  double ms_steps;             /* all outer steps, from events around each replay or batch */
  double ms_guess;             /* network input tiles + forward pass of an attached guess network
                                  (timed outer steps only; 0 without a network) */
  double ms_coarse;            /* two-level coarse correction: restriction, coarse solve, Z_0 x and
                                  r - A Z_0 x (timed outer steps only; 0 for the one-level method) */
  double coarse_bytes;         /* factor and vector bytes one coarse solve reads and writes (the
                                  algorithmic traffic of the block cyclic reduction); 0 without it */
} dd_stats;

/* Fill *p with the defaults: k = 20, ppwl = 10, 2 x 2 uniform subdomains, overlap 1,
   impedance local matrices, linear deflation, FP64 inner, inner_tol 1e-2,
   inner_maxit 100, outer_tol 1e-6, outer_maxit 3000, no restart, nrhs 1, graph replay of
   8 outer steps. */
void dd_default_params(dd_params* p);

/* Build the mesh, the partition, every E_j = Z_j^T B_j Z_j (Sec. 2, eq. 4) and its
   FP64 block factorisation on the device (twisted for linear deflation, one-ended over
   paired rows for Bezier), and allocate all workspaces.  `stream` orders the
   set-up work; the call synchronises it.  Errors: DD_EINVAL (bad parameters,
   reported before allocating), DD_ENOMEM, DD_EHIP, DD_ESINGULAR. */
dd_status dd_setup(const dd_params* p, void* stream, dd_handle** out);

/* z = M^{-1} r = sum_j R_j^T D_j u_j (Sec. 2, eq. 3), every u_j an inexact deflated-GMRES
   solve of the local system with right-hand side R_j r, all subdomains and right-hand
   sides in one launch (with coarse_intervals > 0 the two-level form, see dd_params).
   r, z: device complex128 [nrhs][ndof], must not alias. */
dd_status dd_apply_preconditioner(dd_handle* h, const void* r, void* z, void* stream);

/* Solve A u = f by right-preconditioned FGMRES from u = 0 (Sec. 3).  f, u: device
   complex128 [nrhs][ndof].  stats (host, may be NULL) receives counts.  Returns
   DD_ENOTCONV (u still holds the last iterate) if outer_maxit is reached. */
dd_status dd_solve(dd_handle* h, const void* f, void* u, void* stream, dd_stats* stats);

dd_status dd_destroy(dd_handle* h);
/* Switch graph replay of the outer steps on or off for later dd_solve calls (the
   per-phase event timings of dd_stats are only available with it off).  DD_EINVAL when
   turning it on for a handle with inner_launch DD_INNER_MULTI (its host loop cannot be
   captured). */
dd_status dd_set_graph(dd_handle* h, int use_graph);
/* Autotuner: time candidate launch configurations on this handle's problem with HIP events
   and keep the fastest: threads per subdomain-solve workgroup (256 or 512), launch order
   (largest tile first or natural) and the workgroup count of the outer dot sweep.  With
   cache_path (may be NULL) a line "<signature> | <choice>" is looked up first (signature:
   GPU architecture, grid, partition hash, overlap, local condition, precision, inner_maxit,
   nrhs, restart) and appended after measuring.  Uses the handle's workspaces: do not call
   it while a solve is in flight.  report (may be NULL) receives a text summary.  DD_EINVAL
   for inner_launch DD_INNER_MULTI (it has no launch configuration to tune). */
dd_status dd_autotune(dd_handle* h, const char* cache_path, void* stream, char* report, int report_len);
const char* dd_last_error(void);

int64_t dd_num_dofs(const dd_handle* h);
int dd_num_subdomains(const dd_handle* h);
int dd_num_intervals(const dd_handle* h);
/* Sizes of packed vectors: fine nodes and coarse nodes summed over subdomains. */
int64_t dd_packed_fine_size(const dd_handle* h);
int64_t dd_packed_coarse_size(const dd_handle* h);

/* Host copy of the layout, 12 ints per subdomain (x block index fastest):
   i0, j0, nx, ny (tile), ax, bx, ay, by (overlapping rectangle), mx, my (coarse grid),
   fine offset, coarse offset (offsets fit in int for every supported size). */
dd_status dd_layout(const dd_handle* h, int32_t* out);

/* Host copy of the coefficients of E_j per coarse node (complex128, [nc][K]; K = 9 for
   linear deflation, neighbour (cx+dx, cy+dy) at 3(dy+1) + (dx+1); K = 25 for Bezier,
   neighbour at 5(dy+2) + (dx+2)) and min |pivot| of its block factorisation. */
dd_status dd_coarse_matrix(const dd_handle* h, int j, double* out, double* min_pivot);

/* ---- kernel-level entry points (parity tests, profiling) ------------------------ */

/* w = A v, global FP64 stencil (Sec. 2, eq. 2); one right-hand side. */
dd_status dd_op_global_apply(dd_handle* h, const void* v, void* w, void* stream);
/* w_j = B_j v_j for every subdomain; packed, complex128 (precision 64) or complex64 (32). */
dd_status dd_op_local_apply(dd_handle* h, int precision, const void* v, void* w, void* stream);
/* w_j = P_j B_j v_j (Sec. 2, eq. 4); packed, precision as above. */
dd_status dd_op_deflated_apply(dd_handle* h, int precision, const void* v, void* w, void* stream);
/* t_j = Z_j^T v_j (eq. 5, linear interpolation transpose); complex128 fine -> coarse. */
dd_status dd_op_restrict(dd_handle* h, const void* v, void* t, void* stream);
/* v_j = Z_j y_j; complex128 coarse -> fine. */
dd_status dd_op_prolong(dd_handle* h, const void* y, void* v, void* stream);
/* y_j = E_j^{-1} t_j with the FP64 block factorisation; complex128 coarse vectors. */
dd_status dd_op_coarse_solve(dd_handle* h, const void* t, void* y, void* stream);
/* f_j = R_j r (packed, precision 64 or 32) from global r; one right-hand side. */
dd_status dd_op_gather(dd_handle* h, int precision, const void* r, void* f, void* stream);
/* z = sum_j R_j^T D_j u_j (Boolean partition of unity) from packed u; one right-hand side. */
dd_status dd_op_scatter(dd_handle* h, int precision, const void* u, void* z, void* stream);
/* Batched inexact subdomain solves in the handle's inner precision: packed f [nrhs][nfine]
   -> packed u (recovered local solutions).  guess (packed, same type) may be NULL.
   iters and flags (host int arrays of nrhs * nsub, may be NULL) receive per-solve
   iteration counts and flags (bit 0 guess accepted, bit 1 not converged).  With
   inner_launch DD_INNER_MULTI the solves run in the multi-launch form and guess must be
   NULL (DD_EINVAL otherwise). */
dd_status dd_op_inner_solve(dd_handle* h, const void* f, const void* guess, void* u, int32_t* iters,
                            int32_t* flags, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): dd_op_inner_solve without a guess, with
   every scratch buffer of the subdomain solves -- Krylov bases, R factors and candidate
   coordinates, kept coarse vectors, work tiles, per-solve counts and flags, counters --
   taken from a static device
   array of 64 MiB that each GPU holds from library load until the process ends, instead of
   the handle's workspaces.  Calls nothing that allocates.  f (packed [nrhs][nfine], the
   handle's inner precision) is read in place and must not change until the solves are done;
   u as dd_op_inner_solve.  iters, flags: host int arrays of nsub * nrhs (may be NULL); when
   both are NULL the call only enqueues work on `stream` (nothing synchronises, so it can be
   captured), otherwise it copies them and synchronises.  Every call on one GPU shares the
   array, which keeps the last call's contents (each call clears the counters it needs):
   calls that overlap on one GPU race.  DD_EINVAL for exact local solves or the multi-launch
   form, or when the handle's solves need more than 64 MiB of scratch (the message gives the
   size; it grows with nrhs * nfine * inner_maxit). */
dd_status dd_op_inner_solve_static(dd_handle* h, const void* f, void* u, int32_t* iters, int32_t* flags,
                                   void* stream);

/* ---- two-level method (coarse_intervals > 0) ---------------------------------------- */

/* Coarse unknowns (M - 1)^2 of the global coarse space, 0 for the one-level method. */
int64_t dd_global_coarse_size(const dd_handle* h);
/* Host copy of E_0 = Z_0^T A Z_0 (real: A has Dirichlet conditions on the whole boundary
   and Z_0 is real), 9 doubles per coarse unknown ((M-1)^2 of them, x fastest), neighbour
   (cx+dx, cy+dy) at 3(dy+1) + (dx+1); and the smallest |pivot| met by the block
   inversions of its cyclic reduction.  DD_EINVAL for a one-level handle. */
dd_status dd_global_coarse_matrix(const dd_handle* h, double* out, double* min_pivot);
/* t = Z_0^T r: global complex128 r [ndof] -> coarse complex128 t [(M-1)^2]; one
   right-hand side. */
dd_status dd_op_global_restrict(dd_handle* h, const void* r, void* t, void* stream);
/* y = E_0^{-1} t by the FP64 block cyclic reduction; coarse complex128 vectors. */
dd_status dd_op_global_coarse_solve(dd_handle* h, const void* t, void* y, void* stream);
/* q = Z_0 y and w = r - A q: the coarse correction and the residual the subdomain
   solves of the two-level preconditioner receive.  r, q, w global complex128 [ndof]
   (q, w may be NULL to skip the copy out), y coarse. */
dd_status dd_op_global_correct(dd_handle* h, const void* r, const void* y, void* q, void* w, void* stream);

/* ---- learned initial guess ---------------------------------------------------------
 * The paper's subdomain GMRES starts from zero (Sec. 3).  A guess network maps the
 * right-hand side of a subdomain solve to a starting vector; the solve keeps it only
 * when it lowers the deflated residual, ||P_j (f_j - B_j g)|| < ||P_j f_j|| (Sec. 2,
 * eq. 4), and otherwise starts from zero, so the stopping test (relative to
 * ||P_j f_j||) and the preconditioner's definition are unchanged.
 *
 * Network: a convolutional encoder-decoder on T x T tiles (subdomain tile at the tile
 * origin, zero padding), bf16 weights and activations with fp32 accumulation.
 *   a1 = relu(conv(x)) [c1, T]        a5 = relu(conv(cat(up(a4), a3))) [c2, T/4]
 *   a2 = relu(conv(pool(a1))) [c2, T/2]  a6 = relu(conv(cat(up(a5), a2))) [c1, T/2]
 *   a3 = relu(conv(pool(a2))) [c3, T/4]  a7 = relu(conv(cat(up(a6), a1))) [c1, T]
 *   a4 = relu(conv(pool(a3))) [c4, T/8]  y  = a7 W8 + b8  (1x1, 2 channels)
 * conv = 3x3, zero padding; pool = 2x2 average; up = 2x nearest; cat = channels, first
 * operand first.  Flat parameters (fp32): W1, b1, ..., W8, b8, each C-ordered, a 3x3
 * weight indexed [ky][kx][cin][cout].
 * Tiles are NHWC fp32.  Input channels: Re f, Im f times s = sqrt(n_j) / ||f_j||, the
 * constant k h, and a mask (1 on nodes, -1 on nodes of an impedance side); 0 outside
 * the subdomain.  Output: Re, Im of s u in the same scaling.  Tile b of a handle's
 * batch is right-hand side b / nsub, subdomain b % nsub.
 */
typedef struct dd_net dd_net;

typedef struct {
  int widths[4];               /* c1..c4, multiples of 16, c1 <= 64 (default 16, 32, 64, 64) */
  int tile;                    /* T: 32, 64 or 128 */
  int max_batch;               /* tiles per call */
  int train;                   /* 1: also allocate gradient and optimiser state */
  unsigned long long seed;     /* He-normal initial weights from this seed, zero biases */
} dd_net_params;

/* Per-tile operator description for the training loss: nx, ny of the subdomain tile;
   edges: bit s set when side s (0 left, 1 right, 2 bottom, 3 top) of the tile is an
   edge of the subdomain's cells; robin: bit s set when side s carries the impedance
   condition; kh = k h. */
typedef struct {
  int nx, ny, edges, robin;
  double kh;
} dd_tile_desc;

void dd_net_default_params(dd_net_params* p);
/* Create an inference network (train = 0) from a weights file: 8 bytes "DDHNET01", a
   little-endian uint32 header length, a JSON header with "widths" (4 ints), "tile" and
   "nparams", then nparams little-endian float32 in the flat order above.  tile <= 0 takes
   the header's tile.  The file is read and validated on the host before any device work:
   DD_EWEIGHTS (message says why) when it cannot be read, lacks the magic or a header
   field, has widths the network does not support, a parameter count that differs from
   what its widths need or from the bytes that follow, or a non-finite parameter; then as
   dd_net_create (DD_EINVAL for tile / max_batch, DD_ENOMEM, DD_EHIP).  The weights of the
   guess network are this library's own (the paper has no learned part). */
dd_status dd_net_load(const char* path, int tile, int max_batch, dd_net** out);
/* Allocate a network and its device workspaces.  DD_EINVAL for unsupported sizes. */
dd_status dd_net_create(const dd_net_params* p, dd_net** out);
dd_status dd_net_destroy(dd_net* net);
int64_t dd_net_num_params(const dd_net* net);
/* Host fp32 parameter vector in, or out (n must equal dd_net_num_params).  Setting
   parameters resets the optimiser state.  Both synchronise the default stream. */
dd_status dd_net_set_params(dd_net* net, const float* host, int64_t n);
dd_status dd_net_get_params(const dd_net* net, float* host, int64_t n);
/* y = network(x) for `batch` tiles: x device fp32 [batch][T][T][4], y device fp32
   [batch][T][T][2]. */
dd_status dd_net_forward(dd_net* net, const float* x, int batch, float* y, void* stream);
/* Training loss and its gradient (network built with train = 1).  x as above, t device
   fp32 [batch][T][T][2] (target s u), desc host [batch].  With e = m (y - t) on the tile's
   nodes and B the tile's subdomain operator (Sec. 2, eq. 2, impedance rows per desc):
     loss = mean_b ( w_res ||B e||^2 / ||B t||^2 + w_err ||e||^2 / ||t||^2 ).
   grad (device fp32 [num_params], may be NULL) receives dloss/dparams, which also stays
   in the network for dd_net_adam; *loss (host, may be NULL) the loss.  Synchronises
   `stream`. */
dd_status dd_net_gradient(dd_net* net, const float* x, const float* t, const dd_tile_desc* desc, int batch,
                          double w_res, double w_err, float* grad, double* loss, void* stream);
/* One Adam step (Kingma and Ba, 2015) with the last gradient. */
dd_status dd_net_adam(dd_net* net, double lr, double beta1, double beta2, double eps, void* stream);

/* Attach a network to a handle (NULL detaches): later preconditioner applications and
   solves evaluate it on every subdomain right-hand side and offer the result as the
   initial guess.  The network is borrowed (the caller keeps it alive while attached)
   and must have tile >= every subdomain's nx, ny and max_batch >= nsub * nrhs.
   Attaching allocates nothing.  DD_EINVAL for inner_launch DD_INNER_MULTI. */
dd_status dd_set_guess(dd_handle* h, dd_net* net);
/* Network input tiles of all subdomain solves of global r (device complex128
   [nrhs][ndof]): x device fp32 [nsub * nrhs][T][T][4] and the scales s (device double
   [nsub * nrhs]). */
dd_status dd_tiles(dd_handle* h, const void* r, int tile, float* x, double* scale, void* stream);
/* t = s u as tiles from packed complex128 u [nrhs][nfine] (targets for training). */
dd_status dd_packed_to_tiles(dd_handle* h, const void* u, const double* scale, int tile, float* t, void* stream);
/* Host copy of the per-subdomain tile descriptions (nsub entries). */
dd_status dd_tile_descs(const dd_handle* h, dd_tile_desc* out);
/* Host copies of the per-solve inner iteration counts and flags (bit 0 guess accepted,
   bit 1 not converged) of the last batched subdomain-solve launch of this handle
   (nsub * nrhs entries each, solve rhs * nsub + sub; either pointer may be NULL).
   Synchronises `stream`. */
dd_status dd_last_inner(const dd_handle* h, int32_t* iters, int32_t* flags, void* stream);
/* Copy the j-th outer FGMRES basis vector of the last solve (0 <= j <= its Krylov
   dimension) to v (device complex128 [nrhs][ndof]). */
dd_status dd_outer_basis(dd_handle* h, int j, void* v, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DDHELM_H */
