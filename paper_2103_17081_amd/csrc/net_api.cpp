// C ABI of the learned initial-guess network (dd_net_*): parameters, forward pass,
// training gradient and Adam step, all on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>

#include "net_host.hpp"

namespace ddh {
dd_status fail_msg(dd_status s, const std::string& msg);   // api.cpp
}

namespace {

using ddh::bf16;
using ddh::bf16x8;

#define NET_HIP(expr)                                                                                      \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess)                                                                                   \
      return ddh::fail_msg(e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP,                                 \
                           std::string(#expr) + ": " + hipGetErrorString(e_));                              \
  } while (0)

#define NET_TRY(expr)                 \
  do {                                \
    dd_status s_ = (expr);            \
    if (s_ != DD_OK) return s_;       \
  } while (0)

template <typename T>
dd_status net_alloc(dd_net* n, T** ptr, size_t count) {
  void* q = nullptr;
  NET_HIP(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)));
  n->allocs.push_back(q);
  *ptr = (T*)q;
  return DD_OK;
}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Layer table of the encoder-decoder (see net.hpp) for widths c[0..3].
void build_table(dd_net* n) {
  const int c1 = n->c[0], c2 = n->c[1], c3 = n->c[2], c4 = n->c[3];
  struct Spec { int cin, cinp, cout, level, mode, c1, s0, s1; };
  const Spec sp[ddh::kNetConv] = {
      {ddh::kNetIn, ddh::kNetInP, c1, 0, ddh::kPlain, 0, -1, -1},
      {c1, c1, c2, 1, ddh::kPool, 0, 0, -1},
      {c2, c2, c3, 2, ddh::kPool, 0, 1, -1},
      {c3, c3, c4, 3, ddh::kPool, 0, 2, -1},
      {c4 + c3, c4 + c3, c2, 2, ddh::kUpCat, c4, 3, 2},
      {c2 + c2, c2 + c2, c1, 1, ddh::kUpCat, c2, 4, 1},
      {c1 + c1, c1 + c1, c1, 0, ddh::kUpCat, c1, 5, 0},
  };
  long long po = 0, fo = 0;
  for (int i = 0; i < ddh::kNetConv; ++i) {
    ddh::NetLayer& L = n->nt.l[i];
    L.cin = sp[i].cin;
    L.cinp = sp[i].cinp;
    L.cout = sp[i].cout;
    L.level = sp[i].level;
    L.mode = sp[i].mode;
    L.c1 = sp[i].c1;
    L.src0 = sp[i].s0;
    L.src1 = sp[i].s1;
    L.woff = po;
    po += 9LL * L.cin * L.cout;
    L.boff = po;
    po += L.cout;
    L.ksteps = (9 * L.cinp + 31) / 32;
    L.bksteps = (9 * L.cout + 31) / 32;
    L.ffrag = fo;
    fo += (long long)L.ksteps * (L.cout / 16) * 64;
    L.bfrag = fo;
    if (i > 0) fo += (long long)L.bksteps * (L.cin / 16) * 64;
  }
  n->nt.c1 = c1;
  n->nt.hwoff = po;
  po += 2LL * c1;
  n->nt.hboff = po;
  po += 2;
  n->nparams = po;
  n->nfrag = fo;
}

// Forward product arguments of layer i (input operands from the activations).
ddh::ConvArgs layer_args(const dd_net* n, int i) {
  const ddh::NetLayer& L = n->nt.l[i];
  ddh::ConvArgs a{};
  a.x0 = L.src0 < 0 ? n->x : n->act[L.src0];
  a.x1 = L.src1 < 0 ? nullptr : n->act[L.src1];
  a.wf = n->frags + L.ffrag;
  a.bias = n->params + L.boff;
  a.H = a.W = n->H(L.level);
  a.lw = log2i(a.W);
  a.cinp = L.cinp;
  a.c1 = L.c1;
  a.mode = L.mode;
  a.relu = 1;
  a.ksteps = L.ksteps;
  a.nb = L.cout / 16;
  return a;
}

dd_status prepare(dd_net* n, hipStream_t st) {
  NET_HIP(ddh::launch_net_prepare(n->nt, n->params, n->frags, st));
  return DD_OK;
}

dd_status backward(dd_net* n, int batch, hipStream_t st) {
  const ddh::NetTable& nt = n->nt;
  // head weights and bias
  NET_HIP(ddh::launch_wgrad_reduce(n->part, n->bpart, batch, nt.c1, nt.c1, 2, 1, n->grads + nt.hwoff,
                                   n->grads + nt.hboff, st));
  for (int i = ddh::kNetConv - 1; i >= 0; --i) {
    const ddh::NetLayer& L = nt.l[i];
    ddh::ConvArgs a = layer_args(n, i);
    NET_HIP(ddh::launch_conv_wgrad(a, n->dz[i], L.cout, batch, n->part, n->bpart, st));
    NET_HIP(ddh::launch_wgrad_reduce(n->part, n->bpart, batch, L.cin, L.cinp, L.cout, 9, n->grads + L.woff,
                                     n->grads + L.boff, st));
    if (i == 0) break;
    // data gradient at the layer input: the same product with flipped weights
    ddh::ConvArgs d{};
    d.x0 = n->dz[i];
    d.wf = n->frags + L.bfrag;
    d.out_f = n->dc[i];
    d.H = d.W = n->H(L.level);
    d.lw = log2i(d.W);
    d.cinp = L.cout;
    d.mode = ddh::kPlain;
    d.relu = 0;
    d.ksteps = L.bksteps;
    d.nb = L.cin / 16;
    NET_HIP(ddh::launch_conv(d, batch, st));
    // route into dz of the layer producing activation i-1 (see the layer table)
    const int ti = L.src0;
    const ddh::NetLayer& P = nt.l[ti];
    ddh::RouteArgs r{};
    r.act = n->act[ti];
    r.dz = n->dz[ti];
    r.H = r.W = n->H(P.level);
    r.C = P.cout;
    r.total = (long long)batch * r.H * r.W * r.C;
    if (L.mode == ddh::kUpCat) {
      // input cat(up(a_ti), skip): the first P.cout channels come from a_ti
      r.fine = n->dc[i];
      r.fstride = L.cin;
      r.foff = 0;
    } else {
      // input pool(a_ti); a_ti also feeds the skip half of a decoder layer's input
      int k = -1;
      for (int q = 0; q < ddh::kNetConv; ++q)
        if (nt.l[q].mode == ddh::kUpCat && nt.l[q].src1 == ti) k = q;
      if (k >= 0) {
        r.same = n->dc[k];
        r.sstride = nt.l[k].cin;
        r.soff = nt.l[k].c1;
      }
      r.coarse = n->dc[i];
      r.cstride = L.cin;
    }
    NET_HIP(ddh::launch_route(r, st));
  }
  return DD_OK;
}

}  // namespace

void dd_net::release() {
  for (void* q : allocs) (void)hipFree(q);
  allocs.clear();
}

namespace ddh {

dd_status net_forward(dd_net* n, int batch, hipStream_t st, bool head) {
  for (int i = 0; i < kNetConv; ++i) {
    ConvArgs a = layer_args(n, i);
    a.out_bf = n->act[i];
    NET_HIP(launch_conv(a, batch, st));
  }
  if (!head) return DD_OK;
  HeadArgs h{};
  h.a7 = n->act[kNetConv - 1];
  h.params = n->params;
  h.woff = n->nt.hwoff;
  h.boff = n->nt.hboff;
  h.c1 = n->nt.c1;
  h.T = n->T;
  h.y = n->y;
  h.batch = batch;
  NET_HIP(launch_head(h, st));
  return DD_OK;
}

dd_status net_infer_from(dd_net* n, const TileArgs& ta0, int nsub, int nrhs, hipStream_t st) {
  TileArgs ta = ta0;
  ta.T = n->T;
  ta.xb = n->x;
  ta.xf = nullptr;
  ta.scale = n->scale;
  NET_HIP(launch_tiles(ta, nsub, nrhs, st));
  return net_forward(n, nsub * nrhs, st);
}

}  // namespace ddh

extern "C" {

void dd_net_default_params(dd_net_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->widths[0] = 16;
  p->widths[1] = 32;
  p->widths[2] = 64;
  p->widths[3] = 64;
  p->tile = 64;
  p->max_batch = 256;
  p->train = 0;
  p->seed = 2103170810ULL;
}

dd_status dd_net_create(const dd_net_params* p, dd_net** out) {
  if (!p || !out) return ddh::fail_msg(DD_EINVAL, "null argument");
  *out = nullptr;
  for (int i = 0; i < 4; ++i)
    if (!(p->widths[i] == 16 || p->widths[i] == 32 || p->widths[i] == 64))
      return ddh::fail_msg(DD_EINVAL, "network widths must be 16, 32 or 64");
  if (p->widths[2] != p->widths[3]) return ddh::fail_msg(DD_EINVAL, "network widths c3 and c4 must be equal");
  if (!(p->tile == 32 || p->tile == 64 || p->tile == 128))
    return ddh::fail_msg(DD_EINVAL, "tile must be 32, 64 or 128");
  if (p->max_batch < 1 || p->max_batch > 65535) return ddh::fail_msg(DD_EINVAL, "max_batch must be in [1, 65535]");
  dd_net* n = new dd_net();
  n->p = *p;
  n->T = p->tile;
  n->B = p->max_batch;
  for (int i = 0; i < 4; ++i) n->c[i] = p->widths[i];
  build_table(n);
  auto fin = [&](dd_status s) {
    if (s != DD_OK) {
      n->release();
      delete n;
    }
    return s;
  };
  const size_t B = (size_t)n->B, T2 = (size_t)n->T * n->T;
  dd_status s = DD_OK;
#define NET_A(ptr, cnt) \
  if (s == DD_OK) s = net_alloc(n, &(ptr), (cnt))
  NET_A(n->params, (size_t)n->nparams);
  NET_A(n->frags, (size_t)n->nfrag);
  NET_A(n->x, B * T2 * ddh::kNetInP);
  NET_A(n->y, B * T2 * 2);
  NET_A(n->scale, B);
  for (int i = 0; i < ddh::kNetConv; ++i) {
    const int H = n->H(n->nt.l[i].level);
    NET_A(n->act[i], B * H * H * n->nt.l[i].cout);
  }
  if (p->train) {
    NET_A(n->grads, (size_t)n->nparams);
    NET_A(n->m, (size_t)n->nparams);
    NET_A(n->v, (size_t)n->nparams);
    size_t part = 2 * (size_t)n->nt.c1;
    for (int i = 0; i < ddh::kNetConv; ++i) {
      const ddh::NetLayer& L = n->nt.l[i];
      const int H = n->H(L.level);
      NET_A(n->dz[i], B * H * H * L.cout);
      if (i > 0) NET_A(n->dc[i], B * H * H * L.cin);
      part = std::max(part, (size_t)9 * L.cinp * L.cout);
    }
    NET_A(n->E, B * T2 * 2);
    NET_A(n->R, B * T2 * 2);
    NET_A(n->t, B * T2 * 2);
    NET_A(n->part, B * part);
    NET_A(n->bpart, B * 64);
    NET_A(n->loss, B);
    NET_A(n->desc, B);
  }
#undef NET_A
  if (s != DD_OK) return fin(s);
  if (hipMemset(n->x, 0, B * T2 * ddh::kNetInP * sizeof(bf16)) != hipSuccess ||
      hipMemset(n->y, 0, B * T2 * 2 * sizeof(float)) != hipSuccess)
    return fin(ddh::fail_msg(DD_EHIP, "hipMemset of network buffers failed"));
  if (ddh::configure_net() != hipSuccess) return fin(ddh::fail_msg(DD_EHIP, "configuring network kernels failed"));
  // He-normal initial weights, zero biases
  std::vector<float> w((size_t)n->nparams, 0.0f);
  std::mt19937_64 rng(p->seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int i = 0; i < ddh::kNetConv; ++i) {
    const ddh::NetLayer& L = n->nt.l[i];
    const double sd = std::sqrt(2.0 / (9.0 * L.cin));
    for (long long q = 0; q < 9LL * L.cin * L.cout; ++q) w[L.woff + q] = (float)(sd * nd(rng));
  }
  for (long long q = 0; q < 2LL * n->nt.c1; ++q) w[n->nt.hwoff + q] = (float)(std::sqrt(2.0 / n->nt.c1) * nd(rng));
  *out = n;
  s = dd_net_set_params(n, w.data(), n->nparams);
  if (s != DD_OK) {
    *out = nullptr;
    return fin(s);
  }
  return DD_OK;
}

namespace {

// Value of "key" in a flat JSON object: integers, or an array of integers.
bool json_ints(const std::string& js, const std::string& key, std::vector<long long>& out) {
  const size_t k = js.find("\"" + key + "\"");
  if (k == std::string::npos) return false;
  size_t i = js.find(':', k + key.size() + 2);
  if (i == std::string::npos) return false;
  ++i;
  while (i < js.size() && std::isspace((unsigned char)js[i])) ++i;
  const bool arr = i < js.size() && js[i] == '[';
  if (arr) ++i;
  out.clear();
  while (i < js.size()) {
    while (i < js.size() && std::isspace((unsigned char)js[i])) ++i;
    if (i >= js.size()) return false;
    if (arr && js[i] == ']') break;
    char* end = nullptr;
    const long long v = std::strtoll(js.c_str() + i, &end, 10);
    if (end == js.c_str() + i) return false;
    out.push_back(v);
    i = (size_t)(end - js.c_str());
    while (i < js.size() && std::isspace((unsigned char)js[i])) ++i;
    if (!arr) break;
    if (i < js.size() && js[i] == ',') ++i;
  }
  return !out.empty();
}

}  // namespace

dd_status dd_net_load(const char* path, int tile, int max_batch, dd_net** out) {
  if (!path || !out) return ddh::fail_msg(DD_EINVAL, "null argument");
  *out = nullptr;
  const std::string where = std::string(path) + ": ";
  std::vector<char> data;
  {
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return ddh::fail_msg(DD_EWEIGHTS, where + "cannot open the weights file");
    char buf[1 << 16];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), fp)) > 0) data.insert(data.end(), buf, buf + got);
    std::fclose(fp);
  }
  static const char kMagic[8] = {'D', 'D', 'H', 'N', 'E', 'T', '0', '1'};
  if (data.size() < 12 || std::memcmp(data.data(), kMagic, 8) != 0)
    return ddh::fail_msg(DD_EWEIGHTS, where + "not a guess-network weights file (magic DDHNET01 missing)");
  uint32_t hl = 0;
  for (int b = 0; b < 4; ++b) hl |= (uint32_t)(unsigned char)data[8 + b] << (8 * b);   // little endian
  if ((size_t)hl > data.size() - 12) return ddh::fail_msg(DD_EWEIGHTS, where + "truncated header");
  const std::string head(data.data() + 12, hl);
  std::vector<long long> widths, ftile, np;
  if (!json_ints(head, "widths", widths) || widths.size() != 4 || !json_ints(head, "tile", ftile) ||
      !json_ints(head, "nparams", np))
    return ddh::fail_msg(DD_EWEIGHTS, where + "header lacks widths[4], tile or nparams");
  dd_net probe;   // host-only: the parameter layout of these widths
  for (int i = 0; i < 4; ++i) {
    if (!(widths[i] == 16 || widths[i] == 32 || widths[i] == 64))
      return ddh::fail_msg(DD_EWEIGHTS, where + "network widths must be 16, 32 or 64");
    probe.c[i] = (int)widths[i];
  }
  if (widths[2] != widths[3]) return ddh::fail_msg(DD_EWEIGHTS, where + "network widths c3 and c4 differ");
  build_table(&probe);
  const size_t payload = data.size() - 12 - hl;
  if (np[0] != probe.nparams || payload != (size_t)probe.nparams * sizeof(float))
    return ddh::fail_msg(DD_EWEIGHTS, where + "header says " + std::to_string(np[0]) + " parameters, the widths need " +
                                          std::to_string(probe.nparams) + ", the file holds " +
                                          std::to_string(payload / sizeof(float)));
  std::vector<float> w((size_t)probe.nparams);
  std::memcpy(w.data(), data.data() + 12 + hl, payload);   // little-endian float32 (x86-64 host)
  for (size_t q = 0; q < w.size(); ++q)
    if (!std::isfinite(w[q]))
      return ddh::fail_msg(DD_EWEIGHTS, where + "parameter " + std::to_string(q) + " is not finite");
  dd_net_params p;
  dd_net_default_params(&p);
  for (int i = 0; i < 4; ++i) p.widths[i] = (int)widths[i];
  p.tile = tile > 0 ? tile : (int)ftile[0];
  p.max_batch = max_batch;
  p.train = 0;
  dd_net* n = nullptr;
  dd_status s = dd_net_create(&p, &n);
  if (s != DD_OK) return s;
  s = dd_net_set_params(n, w.data(), (int64_t)w.size());
  if (s != DD_OK) {
    dd_net_destroy(n);
    return s;
  }
  *out = n;
  return DD_OK;
}

dd_status dd_net_destroy(dd_net* n) {
  if (!n) return DD_OK;
  (void)hipDeviceSynchronize();
  n->release();
  delete n;
  return DD_OK;
}

int64_t dd_net_num_params(const dd_net* n) { return n ? n->nparams : 0; }

dd_status dd_net_set_params(dd_net* n, const float* host, int64_t cnt) {
  if (!n || !host) return ddh::fail_msg(DD_EINVAL, "null argument");
  if (cnt != n->nparams) return ddh::fail_msg(DD_EINVAL, "parameter count mismatch");
  NET_HIP(hipMemcpy(n->params, host, (size_t)cnt * sizeof(float), hipMemcpyHostToDevice));
  if (n->m) {
    NET_HIP(hipMemset(n->m, 0, (size_t)cnt * sizeof(float)));
    NET_HIP(hipMemset(n->v, 0, (size_t)cnt * sizeof(float)));
  }
  n->adam_t = 0;
  NET_TRY(prepare(n, nullptr));
  NET_HIP(hipDeviceSynchronize());
  return DD_OK;
}

dd_status dd_net_get_params(const dd_net* n, float* host, int64_t cnt) {
  if (!n || !host) return ddh::fail_msg(DD_EINVAL, "null argument");
  if (cnt != n->nparams) return ddh::fail_msg(DD_EINVAL, "parameter count mismatch");
  NET_HIP(hipDeviceSynchronize());
  NET_HIP(hipMemcpy(host, n->params, (size_t)cnt * sizeof(float), hipMemcpyDeviceToHost));
  return DD_OK;
}

dd_status dd_net_forward(dd_net* n, const float* x, int batch, float* y, void* stream) {
  if (!n || !x || !y) return ddh::fail_msg(DD_EINVAL, "null argument");
  if (batch < 1 || batch > n->B) return ddh::fail_msg(DD_EINVAL, "batch out of range");
  hipStream_t st = (hipStream_t)stream;
  const long long pix = (long long)batch * n->T * n->T;
  NET_HIP(ddh::launch_input_convert(x, n->x, pix, st));
  NET_TRY(ddh::net_forward(n, batch, st));
  NET_HIP(hipMemcpyAsync(y, n->y, (size_t)pix * 2 * sizeof(float), hipMemcpyDeviceToDevice, st));
  return DD_OK;
}

dd_status dd_net_gradient(dd_net* n, const float* x, const float* t, const dd_tile_desc* desc, int batch,
                          double w_res, double w_err, float* grad, double* loss, void* stream) {
  if (!n || !x || !t || !desc) return ddh::fail_msg(DD_EINVAL, "null argument");
  if (!n->grads) return ddh::fail_msg(DD_EINVAL, "network was created without training state");
  if (batch < 1 || batch > n->B) return ddh::fail_msg(DD_EINVAL, "batch out of range");
  if (!(w_res >= 0.0) || !(w_err >= 0.0)) return ddh::fail_msg(DD_EINVAL, "loss weights must be non-negative");
  for (int b = 0; b < batch; ++b)
    if (desc[b].nx < 1 || desc[b].ny < 1 || desc[b].nx > n->T || desc[b].ny > n->T)
      return ddh::fail_msg(DD_EINVAL, "tile description larger than the tile");
  static_assert(sizeof(dd_tile_desc) == sizeof(ddh::TileDescDev), "tile description layout");
  hipStream_t st = (hipStream_t)stream;
  const long long pix = (long long)batch * n->T * n->T;
  NET_HIP(hipMemcpyAsync(n->desc, desc, (size_t)batch * sizeof(dd_tile_desc), hipMemcpyHostToDevice, st));
  NET_HIP(ddh::launch_input_convert(x, n->x, pix, st));
  NET_TRY(ddh::net_forward(n, batch, st, false));
  ddh::HeadArgs h{};
  h.a7 = n->act[ddh::kNetConv - 1];
  h.params = n->params;
  h.woff = n->nt.hwoff;
  h.boff = n->nt.hboff;
  h.c1 = n->nt.c1;
  h.T = n->T;
  h.y = n->y;
  h.t = t;
  h.desc = n->desc;
  h.w_res = w_res;
  h.w_err = w_err;
  h.batch = batch;
  h.E = n->E;
  h.R = n->R;
  h.dz7 = n->dz[ddh::kNetConv - 1];
  h.part = n->part;
  h.bpart = n->bpart;
  h.loss = n->loss;
  NET_HIP(ddh::launch_head(h, st));
  NET_TRY(backward(n, batch, st));
  if (grad) NET_HIP(hipMemcpyAsync(grad, n->grads, (size_t)n->nparams * sizeof(float), hipMemcpyDeviceToDevice, st));
  std::vector<double> lp(batch);
  NET_HIP(hipMemcpyAsync(lp.data(), n->loss, (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, st));
  NET_HIP(hipStreamSynchronize(st));
  if (loss) {
    double s = 0.0;
    for (double v : lp) s += v;
    *loss = s / batch;
  }
  return DD_OK;
}

dd_status dd_net_adam(dd_net* n, double lr, double beta1, double beta2, double eps, void* stream) {
  if (!n) return ddh::fail_msg(DD_EINVAL, "null argument");
  if (!n->grads) return ddh::fail_msg(DD_EINVAL, "network was created without training state");
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return ddh::fail_msg(DD_EINVAL, "invalid Adam hyper-parameters");
  hipStream_t st = (hipStream_t)stream;
  ++n->adam_t;
  const double c1 = 1.0 - std::pow(beta1, (double)n->adam_t), c2 = 1.0 - std::pow(beta2, (double)n->adam_t);
  NET_HIP(ddh::launch_adam(n->params, n->grads, n->m, n->v, n->nparams, (float)lr, (float)beta1, (float)beta2,
                           (float)eps, (float)c1, (float)c2, st));
  NET_TRY(prepare(n, st));
  return DD_OK;
}

}  // extern "C"
