// Learned initial guess for the subdomain solves: a small convolutional
// encoder-decoder on zero-padded T x T tiles, evaluated and trained with bf16 MFMA
// products (fp32 accumulation).  The paper's subdomain solver starts from a zero
// guess (Sec. 3); the guess produced here only replaces that start when it lowers the
// deflated residual, so the preconditioner it feeds is still the paper's.
//
// Network (widths c1..c4, all multiples of 16; "conv" = 3x3, zero padding, stride 1):
//   a1 = relu(conv(x))                 c1 @ T        a5 = relu(conv(cat(up(a4), a3)))  c2 @ T/4
//   a2 = relu(conv(pool(a1)))          c2 @ T/2      a6 = relu(conv(cat(up(a5), a2)))  c1 @ T/2
//   a3 = relu(conv(pool(a2)))          c3 @ T/4      a7 = relu(conv(cat(up(a6), a1)))  c1 @ T
//   a4 = relu(conv(pool(a3)))          c4 @ T/8      y  = a7 W8 + b8 (1x1)             2  @ T
// pool = 2x2 average, up = 2x nearest.  Tensors are NHWC.  The flat parameter vector
// holds W1, b1, ..., W8, b8; a 3x3 weight is indexed [ky][kx][cin][cout].
//
// Input channels: Re f, Im f of the local right-hand side times sqrt(n_j)/||f||, the
// constant k h, and a boundary mask (1 on nodes, -1 on nodes of an impedance side);
// all four are 0 outside the subdomain.  Output: Re, Im of the guess in the same
// scaling.  The network input is stored with 8 channels (4..7 zero) so that every
// layer's input has a multiple of 8 channels.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace ddh {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNetIn = 4;
constexpr int kNetInP = 8;
constexpr int kNetOut = 2;
constexpr int kNetConv = 7;          // 3x3 layers; the 1x1 head follows
constexpr int kNetThreads = 256;

enum ConvMode { kPlain = 0, kPool = 1, kUpCat = 2 };

struct NetLayer {
  int cin, cinp, cout;   // input channels (real / stored), output channels
  int level;             // resolution T >> level of input and output
  int mode, c1;          // input transform; kUpCat: channels from the low-resolution operand
  int src0, src1;        // activation index of the operands (-1: network input)
  long long woff, boff;  // parameter offsets (floats)
  long long ffrag, bfrag;  // offsets (bf16x8 units) of forward / data-gradient fragments
  int ksteps, bksteps;   // 32-wide k steps: forward 9 cinp, data gradient 9 cout
};

struct NetTable {
  NetLayer l[kNetConv];
  int c1;                // head input channels
  long long hwoff, hboff;
};

// Per-tile description used by the loss: subdomain size, which sides are cell edges
// of the subdomain (bit 0 left, 1 right, 2 bottom, 3 top), which are impedance sides
// (same bits), and k h.
struct TileDescDev {
  int nx, ny, edges, robin;
  double kh;
};

// One 3x3 product (forward, or data gradient with the flipped weights).
struct ConvArgs {
  const bf16* x0;        // kPlain: input [B][H][W][cinp]; kPool: [B][2H][2W][cinp]; kUpCat: [B][H/2][W/2][c1]
  const bf16* x1;        // kUpCat: skip operand [B][H][W][cinp - c1]
  const bf16x8* wf;      // weight fragments [ksteps][NB][64 lanes]
  const float* bias;     // [NB*16] or null
  bf16* out_bf;          // [B][H][W][NB*16] (bf16) or null
  float* out_f;          // [B][H][W][NB*16] (fp32) or null
  int H, W, lw;          // lw = log2(W)
  int cinp, c1, mode, relu, ksteps, nb;
};

// Route the data gradients of one level into the gradient at a layer output:
// dz = (upsum(fine[:, foff:foff+C]) + same[:, soff:soff+C] + 0.25 up(coarse)) * (act > 0),
// each term optional.
struct RouteArgs {
  const float* fine; int fstride, foff;
  const float* same; int sstride, soff;
  const float* coarse; int cstride;
  const bf16* act;
  bf16* dz;
  int H, W, C;
  long long total;       // B * H * W * C
};

struct HeadArgs {
  const bf16* a7;
  const float* params;
  long long woff, boff;
  int c1, T;
  float* y;              // [B][T][T][2]
  // training
  const float* t;        // targets [B][T][T][2] or null (inference)
  const TileDescDev* desc;
  double w_res, w_err;
  int batch;
  float* E;              // scratch [B][T][T][2]
  float* R;              // scratch [B][T][T][2]
  bf16* dz7;             // [B][T][T][c1]
  float* part;           // [B][c1][2] weight partials
  float* bpart;          // [B][2] bias partials
  double* loss;          // [B]
};

struct TileArgs {
  const SubDesc* subs;
  Consts cs;
  const cplx<double>* r;     // global vectors [nrhs][ndof], advanced by (*jdev) * rslot if jdev
  long long rstride;
  const int* jdev;
  long long rslot;
  const int* done;
  int T;
  bf16* xb;                  // [B][T][T][8] or null
  float* xf;                 // [B][T][T][4] or null
  double* scale;             // [B] sqrt(n_j) / ||f||  (0 for a zero right-hand side)
};

hipError_t launch_net_prepare(const NetTable& nt, const float* params, bf16x8* frags, hipStream_t st);
hipError_t launch_conv(const ConvArgs& a, int batch, hipStream_t st);
size_t conv_lds_bytes(int H, int W, int cinp, int nb, int ksteps);
hipError_t launch_conv_wgrad(const ConvArgs& a, const bf16* dz, int cout, int batch, float* part, float* bpart,
                             hipStream_t st);
size_t wgrad_lds_bytes(int H, int W, int cinp, int cout);
hipError_t launch_wgrad_reduce(const float* part, const float* bpart, int batch, int cin, int cinp, int cout,
                               int taps, float* gW, float* gb, hipStream_t st);
hipError_t launch_route(const RouteArgs& a, hipStream_t st);
hipError_t launch_head(const HeadArgs& a, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st);
hipError_t launch_input_convert(const float* xf, bf16* xb, long long pixels, hipStream_t st);
hipError_t launch_tiles(const TileArgs& a, int nsub, int nrhs, hipStream_t st);
hipError_t launch_packed_to_tiles(const SubDesc* subs, int nsub, int nrhs, long long nfine,
                                  const cplx<double>* u, const double* scale, int T, float* t, hipStream_t st);
hipError_t configure_net();

}  // namespace ddh
