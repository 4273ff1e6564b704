// Host side of the learned initial guess: the network object behind the dd_net C ABI.
#pragma once

#include <vector>

#include "ddhelm.h"
#include "net.hpp"

struct dd_net {
  dd_net_params p{};
  int T = 0, B = 0;
  int c[4] = {};
  ddh::NetTable nt{};
  long long nparams = 0, nfrag = 0;
  // device
  float* params = nullptr;
  ddh::bf16x8* frags = nullptr;
  ddh::bf16* x = nullptr;            // [B][T][T][8]
  ddh::bf16* act[ddh::kNetConv] = {};
  float* y = nullptr;                // [B][T][T][2]
  double* scale = nullptr;           // [B]
  // training
  float* grads = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  ddh::bf16* dz[ddh::kNetConv] = {};
  float* dc[ddh::kNetConv] = {};     // data gradient at the input of layer i (i >= 1)
  float* E = nullptr;
  float* R = nullptr;
  float* t = nullptr;
  float* part = nullptr;
  float* bpart = nullptr;
  double* loss = nullptr;
  ddh::TileDescDev* desc = nullptr;
  long long adam_t = 0;
  std::vector<void*> allocs;

  int H(int level) const { return T >> level; }
  void release();
};

namespace ddh {

// Network input tiles of the solves of one preconditioner application, the forward
// pass, and the guess tiles in net->y (all on `st`).
dd_status net_infer_from(dd_net* net, const TileArgs& ta, int nsub, int nrhs, hipStream_t st);
// The forward pass on net->x for `batch` tiles, output in net->y.
dd_status net_forward(dd_net* net, int batch, hipStream_t st, bool head = true);

}  // namespace ddh
