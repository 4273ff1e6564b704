// Kernels of the learned initial guess (network layout and scaling in net.hpp).
//
// 3x3 layers are implicit GEMMs on v_mfma_f32_16x16x32_bf16: a workgroup stages a
// band of image rows (plus a one-pixel halo) of the layer input in LDS, applying the
// layer's input transform on the way (2x2 average pooling, or nearest upsampling of
// one operand concatenated with a skip operand), and each wave multiplies 16-pixel
// fragments of the staged band by pre-arranged weight fragments.  The data gradient
// of a layer is the same product with the weights flipped in space and transposed in
// channels; the weight gradient reduces im2col(input)^T dz over the pixels of a tile,
// one partial per tile, summed in a second kernel in a fixed order.
//
// MFMA operand layout (16x16x32): lane l supplies row l % 16 of A and column l % 16
// of B over the same 8 reduction indices (8 (l / 16) + e within the 32-wide step);
// lane l receives rows 4 (l / 16) + i, i < 4, of column l % 16 of the product.
#include <algorithm>

#include "net.hpp"
#include "stencil.hpp"

namespace ddh {

namespace {

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int i = 0; i < 8; ++i) z[i] = (bf16)0.0f;
  return z;
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 8 consecutive input channels (from ch) of layer-input pixel (y, x) of tile b.
__device__ __forceinline__ bf16x8 load_input(const ConvArgs& a, int b, int y, int x, int ch) {
  const int H = a.H, W = a.W;
  if (a.mode == kPlain) return *(const bf16x8*)(a.x0 + (((size_t)b * H + y) * W + x) * a.cinp + ch);
  if (a.mode == kPool) {
    const int W2 = 2 * W;
    const bf16* base = a.x0 + (((size_t)b * 2 * H + 2 * y) * W2 + 2 * x) * a.cinp + ch;
    const bf16x8 v00 = *(const bf16x8*)base;
    const bf16x8 v01 = *(const bf16x8*)(base + a.cinp);
    const bf16x8 v10 = *(const bf16x8*)(base + (size_t)W2 * a.cinp);
    const bf16x8 v11 = *(const bf16x8*)(base + (size_t)W2 * a.cinp + a.cinp);
    bf16x8 o;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      o[i] = (bf16)(0.25f * (((float)v00[i] + (float)v01[i]) + ((float)v10[i] + (float)v11[i])));
    return o;
  }
  if (ch < a.c1) {
    const int Hl = H >> 1, Wl = W >> 1;
    return *(const bf16x8*)(a.x0 + (((size_t)b * Hl + (y >> 1)) * Wl + (x >> 1)) * a.c1 + ch);
  }
  const int cs = a.cinp - a.c1;
  return *(const bf16x8*)(a.x1 + (((size_t)b * H + y) * W + x) * cs + (ch - a.c1));
}

constexpr int kStageBatch = 8;   // staging loads each thread keeps in flight

// Rows y0-1 .. y0+rows of tile b, columns -1 .. W, into LDS (pixel stride cinp + 8).
// Each thread issues kStageBatch loads before storing any, so the band arrives in a few
// memory latencies rather than one per unit.
__device__ __forceinline__ void stage_input(const ConvArgs& a, int b, int y0, int rows, bf16* lds) {
  const int W = a.W, cg = a.cinp >> 3, ps = a.cinp + 8, W2 = W + 2;
  const int units = (rows + 2) * W2 * cg;
  const int nt = blockDim.x;
  for (int u0 = threadIdx.x; u0 < units; u0 += nt * kStageBatch) {
    bf16x8 v[kStageBatch];
#pragma unroll
    for (int q = 0; q < kStageBatch; ++q) {
      const int u = u0 + q * nt;
      v[q] = zero8();
      if (u < units) {
        const int g = u % cg, pc = u / cg;
        const int c = pc % W2, r = pc / W2;
        const int y = y0 - 1 + r, x = c - 1;
        if (y >= 0 && y < a.H && x >= 0 && x < W) v[q] = load_input(a, b, y, x, g * 8);
      }
    }
#pragma unroll
    for (int q = 0; q < kStageBatch; ++q) {
      const int u = u0 + q * nt;
      if (u < units) {
        const int g = u % cg, pc = u / cg;
        *(bf16x8*)(lds + (size_t)pc * ps + g * 8) = v[q];
      }
    }
  }
}

// n bf16x8 values from global to LDS, kStageBatch loads in flight per thread.
__device__ __forceinline__ void stage_copy(const bf16x8* __restrict__ src, bf16x8* dst, int n) {
  const int nt = blockDim.x;
  for (int u0 = threadIdx.x; u0 < n; u0 += nt * kStageBatch) {
    bf16x8 v[kStageBatch];
#pragma unroll
    for (int q = 0; q < kStageBatch; ++q) v[q] = u0 + q * nt < n ? src[u0 + q * nt] : zero8();
#pragma unroll
    for (int q = 0; q < kStageBatch; ++q)
      if (u0 + q * nt < n) dst[u0 + q * nt] = v[q];
  }
}

}  // namespace

// LDS of one 3x3 product with MF fragments per wave: the staged input band (rounded up
// to 16 bytes) followed by all weight fragments of the layer.
static size_t conv_lds_bytes_mf(int H, int W, int cinp, int nb, int ksteps, int mf) {
  const int np = std::min(64 * mf, H * W);
  const int rows = (np + W - 1) / W;
  const size_t in = ((size_t)(rows + 2) * (W + 2) * (cinp + 8) * sizeof(bf16) + 15) & ~size_t(15);
  return in + (size_t)ksteps * nb * 64 * sizeof(bf16x8);
}

// Fragments per wave: 4 unless that band plus the weights exceed the LDS.
static int conv_mf(int H, int W, int cinp, int nb, int ksteps) {
  if (nb >= 8) return 2;
  return conv_lds_bytes_mf(H, W, cinp, nb, ksteps, 4) <= 160 * 1024 ? 4 : 2;
}

size_t conv_lds_bytes(int H, int W, int cinp, int nb, int ksteps) {
  return conv_lds_bytes_mf(H, W, cinp, nb, ksteps, conv_mf(H, W, cinp, nb, ksteps));
}

// out[p][co] = bias[co] + sum_{tap, ci} in[p + off(tap)][ci] W[tap][ci][co]   (+ relu)
// Grid: (ceil(H W / (64 MF)), batch); 256 threads; wave w owns fragments w + 4 f.
template <int NB, int MF>
__global__ void __launch_bounds__(kNetThreads) conv3x3_kernel(ConvArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  bf16* lds = (bf16*)smem;
  const int b = blockIdx.y;
  const int W = a.W, npix = a.H * W;
  const int p0 = blockIdx.x * (64 * MF);
  const int np = min(64 * MF, npix - p0);
  const int y0 = p0 >> a.lw, rows = ((p0 + np - 1) >> a.lw) - y0 + 1;
  stage_input(a, b, y0, rows, lds);
  // all weight fragments of the layer, after the input band (whose LDS size is that of
  // the first block, the largest)
  const int rows0 = (min(64 * MF, npix) + W - 1) / W;
  bf16x8* lwf = (bf16x8*)(smem + ((((size_t)(rows0 + 2) * (W + 2) * (a.cinp + 8) * sizeof(bf16)) + 15) & ~size_t(15)));
  stage_copy(a.wf, lwf, a.ksteps * NB * 64);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
  const int ps = a.cinp + 8, W2 = W + 2;
  f32x4 acc[MF][NB];
  int pofs[MF];
#pragma unroll
  for (int f = 0; f < MF; ++f) {
#pragma unroll
    for (int n = 0; n < NB; ++n) acc[f][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int p = p0 + (wave + 4 * f) * 16 + lr;
    const int py = p >> a.lw, px = p & (W - 1);
    pofs[f] = ((py - y0 + 1) * W2 + px + 1) * ps;
  }
  for (int ks = 0; ks < a.ksteps; ++ks) {
    const int k0 = ks * 32 + lg * 8;
    const int tap = k0 / a.cinp, ch = k0 - tap * a.cinp;
    const bool tv = tap < 9;
    const int toff = tv ? ((tap / 3 - 1) * W2 + (tap % 3 - 1)) * ps + ch : 0;
    bf16x8 wv[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) wv[n] = lwf[(ks * NB + n) * 64 + lane];
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      if ((wave + 4 * f) * 16 < np) {
        const bf16x8 xv = tv ? *(const bf16x8*)(lds + pofs[f] + toff) : zero8();
#pragma unroll
        for (int n = 0; n < NB; ++n) acc[f][n] = mfma(wv[n], xv, acc[f][n]);
      }
    }
  }
  constexpr int C = NB * 16;
#pragma unroll
  for (int f = 0; f < MF; ++f) {
    if ((wave + 4 * f) * 16 >= np) continue;
    const size_t p = (size_t)b * npix + p0 + (wave + 4 * f) * 16 + lr;
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      const int co = n * 16 + 4 * lg;
      float o[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        o[i] = acc[f][n][i] + (a.bias ? a.bias[co + i] : 0.0f);
        if (a.relu) o[i] = fmaxf(o[i], 0.0f);
      }
      if (a.out_bf) {
        bf16x4 v;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = (bf16)o[i];
        *(bf16x4*)(a.out_bf + p * C + co) = v;
      } else {
        *(f32x4*)(a.out_f + p * C + co) = f32x4{o[0], o[1], o[2], o[3]};
      }
    }
  }
}

hipError_t launch_conv(const ConvArgs& a, int batch, hipStream_t st) {
  const int npix = a.H * a.W;
  const int mf = conv_mf(a.H, a.W, a.cinp, a.nb, a.ksteps);
  const dim3 grid((npix + 64 * mf - 1) / (64 * mf), batch);
  const size_t lds = conv_lds_bytes_mf(a.H, a.W, a.cinp, a.nb, a.ksteps, mf);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (mf == 4) {
    switch (a.nb) {
      case 1: hipLaunchKernelGGL((conv3x3_kernel<1, 4>), grid, dim3(kNetThreads), lds, st, a); break;
      case 2: hipLaunchKernelGGL((conv3x3_kernel<2, 4>), grid, dim3(kNetThreads), lds, st, a); break;
      case 4: hipLaunchKernelGGL((conv3x3_kernel<4, 4>), grid, dim3(kNetThreads), lds, st, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.nb) {
      case 1: hipLaunchKernelGGL((conv3x3_kernel<1, 2>), grid, dim3(kNetThreads), lds, st, a); break;
      case 2: hipLaunchKernelGGL((conv3x3_kernel<2, 2>), grid, dim3(kNetThreads), lds, st, a); break;
      case 4: hipLaunchKernelGGL((conv3x3_kernel<4, 2>), grid, dim3(kNetThreads), lds, st, a); break;
      case 8: hipLaunchKernelGGL((conv3x3_kernel<8, 2>), grid, dim3(kNetThreads), lds, st, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// ---- weight gradient ----------------------------------------------------------------

namespace {
constexpr int kWgPix = 256;                 // pixels staged per pass
constexpr int kWgDzStride = kWgPix + 8;     // LDS row stride of the transposed dz block
constexpr int kWgTilesPerWave = 8;          // 16x16 output tiles per wave
}  // namespace

size_t wgrad_lds_bytes(int H, int W, int cinp, int cout) {
  const int np = std::min(kWgPix, H * W);
  const int rows = (np + W - 1) / W;
  const size_t in = (size_t)(rows + 2) * (W + 2) * (cinp + 8) * sizeof(bf16);
  return in + (size_t)cout * kWgDzStride * sizeof(bf16) + kNetThreads * sizeof(float);
}

// part[b][tap cinp + ci][co] = sum_p in[p + off(tap)][ci] dz[p][co]   over the pixels of tile b;
// bpart[b][co] = sum_p dz[p][co] (workgroups with blockIdx.x == 0).
// Grid: (ceil(NB KC / 32), batch); wave w of chunk c owns output tiles 32 c + 8 w + q.
__global__ void __launch_bounds__(kNetThreads) conv3x3_wgrad_kernel(ConvArgs a, const bf16* __restrict__ dz,
                                                                     int cout, float* __restrict__ part,
                                                                     float* __restrict__ bpart) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.y;
  const int W = a.W, npix = a.H * W, W2 = W + 2, ps = a.cinp + 8;
  const int npass = std::min(kWgPix, npix);
  const int rows_max = (npass + W - 1) / W;
  bf16* lin = (bf16*)smem;
  bf16* ldz = lin + (size_t)(rows_max + 2) * W2 * ps;
  float* lred = (float*)(ldz + (size_t)cout * kWgDzStride);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
  const int Kp = 9 * a.cinp, KC = (Kp + 15) / 16, NB = cout / 16, ntile = NB * KC;
  const int obase = blockIdx.x * (4 * kWgTilesPerWave) + wave * kWgTilesPerWave;
  f32x4 acc[kWgTilesPerWave];
#pragma unroll
  for (int q = 0; q < kWgTilesPerWave; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool do_bias = blockIdx.x == 0;
  const int bco = tid % cout, bstripe = kNetThreads / cout;
  float bsum = 0.0f;
  for (int p0 = 0; p0 < npix; p0 += kWgPix) {
    const int np = std::min(kWgPix, npix - p0);
    const int y0 = p0 >> a.lw, rows = ((p0 + np - 1) >> a.lw) - y0 + 1;
    const int npad = (np + 31) & ~31;
    __syncthreads();
    stage_input(a, b, y0, rows, lin);
    for (int e = tid; e < cout * npad; e += kNetThreads) {
      const int co = e / npad, q = e - co * npad;
      ldz[co * kWgDzStride + q] = q < np ? dz[((size_t)b * npix + p0 + q) * cout + co] : (bf16)0.0f;
    }
    __syncthreads();
    if (do_bias)
      for (int q = tid / cout; q < np; q += bstripe) bsum += (float)ldz[bco * kWgDzStride + q];
#pragma unroll
    for (int q = 0; q < kWgTilesPerWave; ++q) {
      const int o = obase + q;
      if (o >= ntile) break;
      const int nb = o / KC, kc = o - nb * KC;
      const int k = kc * 16 + lr;
      const int tap = k / a.cinp, ci = k - tap * a.cinp;
      const bool kv = tap < 9;
      const int toff = kv ? ((tap / 3 - 1) * W2 + (tap % 3 - 1)) * ps + ci : 0;
      const bf16* dzrow = ldz + (nb * 16 + lr) * kWgDzStride;
      for (int s = 0; s < npad; s += 32) {
        const bf16x8 av = *(const bf16x8*)(dzrow + s + 8 * lg);
        bf16x8 bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int qq = s + 8 * lg + e;
          bf16 v = (bf16)0.0f;
          if (kv && qq < np) {
            const int p = p0 + qq, py = p >> a.lw, px = p & (W - 1);
            v = lin[((py - y0 + 1) * W2 + px + 1) * ps + toff];
          }
          bv[e] = v;
        }
        acc[q] = mfma(av, bv, acc[q]);
      }
    }
  }
  // lane holds rows co = nb 16 + 4 lg + i of column k = kc 16 + lr
#pragma unroll
  for (int q = 0; q < kWgTilesPerWave; ++q) {
    const int o = obase + q;
    if (o >= ntile) break;
    const int nb = o / KC, kc = o - nb * KC;
    const int k = kc * 16 + lr;
    if (k < Kp) {
#pragma unroll
      for (int i = 0; i < 4; ++i) part[((size_t)b * Kp + k) * cout + nb * 16 + 4 * lg + i] = acc[q][i];
    }
  }
  if (do_bias) {
    lred[tid] = bsum;
    __syncthreads();
    if (tid < cout) {
      float s = 0.0f;
      for (int j = tid; j < kNetThreads; j += cout) s += lred[j];
      bpart[(size_t)b * cout + tid] = s;
    }
  }
}

hipError_t launch_conv_wgrad(const ConvArgs& a, const bf16* dz, int cout, int batch, float* part, float* bpart,
                             hipStream_t st) {
  const int Kp = 9 * a.cinp, KC = (Kp + 15) / 16, ntile = (cout / 16) * KC;
  const dim3 grid((ntile + 4 * kWgTilesPerWave - 1) / (4 * kWgTilesPerWave), batch);
  hipLaunchKernelGGL(conv3x3_wgrad_kernel, grid, dim3(kNetThreads), wgrad_lds_bytes(a.H, a.W, a.cinp, cout), st, a,
                     dz, cout, part, bpart);
  return hipGetLastError();
}

// gW[(tap cin + ci) cout + co] = sum_b part[b][tap cinp + ci][co];  gb[co] = sum_b bpart[b][co].
// `taps` is 9 for 3x3 layers and 1 for the head (whose partials are [b][cin][cout]).
__global__ void wgrad_reduce_kernel(const float* __restrict__ part, const float* __restrict__ bpart, int batch,
                                    int cin, int cinp, int cout, int taps, float* __restrict__ gW,
                                    float* __restrict__ gb) {
  const long long nW = (long long)taps * cin * cout;
  const long long Kp = (long long)taps * cinp;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nW + cout;
       idx += (long long)gridDim.x * blockDim.x) {
    float s = 0.0f;
    if (idx < nW) {
      const int co = (int)(idx % cout);
      const long long r = idx / cout;
      const int ci = (int)(r % cin), tap = (int)(r / cin);
      const long long k = (long long)tap * cinp + ci;
      for (int b = 0; b < batch; ++b) s += part[((long long)b * Kp + k) * cout + co];
      gW[idx] = s;
    } else {
      const int co = (int)(idx - nW);
      for (int b = 0; b < batch; ++b) s += bpart[(long long)b * cout + co];
      gb[co] = s;
    }
  }
}

hipError_t launch_wgrad_reduce(const float* part, const float* bpart, int batch, int cin, int cinp, int cout,
                               int taps, float* gW, float* gb, hipStream_t st) {
  const long long n = (long long)taps * cin * cout + cout;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(blocks), dim3(256), 0, st, part, bpart, batch, cin, cinp, cout, taps,
                     gW, gb);
  return hipGetLastError();
}

// ---- weight fragments ------------------------------------------------------------

// Forward fragment e of lane l at (ks, nb): W[tap][ci][co] with k = 32 ks + 8 (l/16) + e =
// tap cinp + ci and co = 16 nb + l % 16 (0 for padded channels and taps >= 9).
// Data-gradient fragment: k' = tap' cout + co, n' = ci:  W[8 - tap'][ci][co].
__global__ void net_prepare_kernel(NetTable nt, const float* __restrict__ params, bf16x8* __restrict__ frags) {
  for (int li = 0; li < kNetConv; ++li) {
    const NetLayer& L = nt.l[li];
    const int nbf = L.cout / 16, nbb = L.cin / 16;
    const long long nf = (long long)L.ksteps * nbf * 64;
    const long long nbk = (li == 0) ? 0 : (long long)L.bksteps * nbb * 64;
    for (long long u = blockIdx.x * (long long)blockDim.x + threadIdx.x; u < nf + nbk;
         u += (long long)gridDim.x * blockDim.x) {
      bf16x8 v;
      if (u < nf) {
        const int lane = (int)(u % 64);
        const long long r = u / 64;
        const int nb = (int)(r % nbf), ks = (int)(r / nbf);
        const int co = nb * 16 + lane % 16;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = ks * 32 + 8 * (lane / 16) + e;
          const int tap = k / L.cinp, ci = k - tap * L.cinp;
          float w = 0.0f;
          if (tap < 9 && ci < L.cin) w = params[L.woff + ((long long)tap * L.cin + ci) * L.cout + co];
          v[e] = (bf16)w;
        }
        frags[L.ffrag + u] = v;
      } else {
        const long long ub = u - nf;
        const int lane = (int)(ub % 64);
        const long long r = ub / 64;
        const int nb = (int)(r % nbb), ks = (int)(r / nbb);
        const int ci = nb * 16 + lane % 16;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = ks * 32 + 8 * (lane / 16) + e;
          const int tap = k / L.cout, co = k - tap * L.cout;
          float w = 0.0f;
          if (tap < 9) w = params[L.woff + ((long long)(8 - tap) * L.cin + ci) * L.cout + co];
          v[e] = (bf16)w;
        }
        frags[L.bfrag + ub] = v;
      }
    }
  }
}

hipError_t launch_net_prepare(const NetTable& nt, const float* params, bf16x8* frags, hipStream_t st) {
  hipLaunchKernelGGL(net_prepare_kernel, dim3(256), dim3(256), 0, st, nt, params, frags);
  return hipGetLastError();
}

// ---- gradient routing between levels ----------------------------------------------------

__global__ void route_kernel(RouteArgs a) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < a.total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(idx % a.C);
    const long long pix = idx / a.C;
    const int x = (int)(pix % a.W);
    const long long r = pix / a.W;
    const int y = (int)(r % a.H);
    const long long b = r / a.H;
    float g = 0.0f;
    if (a.fine) {
      const int Wf = 2 * a.W;
      const float* f = a.fine + (((b * 2 * a.H) + 2 * y) * Wf + 2 * x) * a.fstride + a.foff + c;
      g += (f[0] + f[a.fstride]) + (f[(long long)Wf * a.fstride] + f[(long long)Wf * a.fstride + a.fstride]);
    }
    if (a.same) g += a.same[pix * a.sstride + a.soff + c];
    if (a.coarse) {
      const int Wc = a.W >> 1;
      g += 0.25f * a.coarse[((b * (a.H >> 1) + (y >> 1)) * Wc + (x >> 1)) * a.cstride + c];
    }
    a.dz[idx] = (float)a.act[idx] > 0.0f ? (bf16)g : (bf16)0.0f;
  }
}

hipError_t launch_route(const RouteArgs& a, hipStream_t st) {
  const int blocks = (int)std::min<long long>((a.total + 255) / 256, 8192);
  hipLaunchKernelGGL(route_kernel, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---- head: 1x1 output layer, loss, and the first backward steps ----------------------------

namespace {

__device__ __forceinline__ double block_sum_d(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kNetThreads / kWave; ++w) s += red[w];
  return s;
}

// (B v)_p for node p = (li, lj) of the tile operator, v read through `get` (complex).
template <typename Get>
__device__ __forceinline__ cplx<float> tile_apply(const cplx<float>* tab, const TileDescDev& d, int li, int lj,
                                                  Get get) {
  const int xc = (li == 0 && (d.edges & 1)) ? 0 : ((li == d.nx - 1 && (d.edges & 2)) ? 2 : 1);
  const int yc = (lj == 0 && (d.edges & 4)) ? 0 : ((lj == d.ny - 1 && (d.edges & 8)) ? 2 : 1);
  const cplx<float>* c = tab + kStencilPts * (3 * yc + xc);
  cplx<float> acc = c[kC] * get(li, lj);
  if (li > 0) acc = cfma(c[kW], get(li - 1, lj), acc);
  if (li < d.nx - 1) acc = cfma(c[kE], get(li + 1, lj), acc);
  if (lj > 0) {
    acc = cfma(c[kS], get(li, lj - 1), acc);
    if (li > 0) acc = cfma(c[kSW], get(li - 1, lj - 1), acc);
  }
  if (lj < d.ny - 1) {
    acc = cfma(c[kN], get(li, lj + 1), acc);
    if (li < d.nx - 1) acc = cfma(c[kNE], get(li + 1, lj + 1), acc);
  }
  return acc;
}

}  // namespace

// One workgroup per tile.  Inference: y = a7 W8 + b8.  Training additionally forms, with
// e = m (y - t) and r = B e (B the tile's subdomain operator, m its node mask),
//   loss_b = w_res ||r||^2 / ||B t||^2 + w_err ||e||^2 / ||m t||^2,
//   dL/dy  = (w_res 2 B^H r / ||B t||^2 + w_err 2 e / ||m t||^2) / batch   on nodes,
// then the head's weight and bias partials and dz7 = (dL/dy W8^T) * (a7 > 0).
template <int C>
__global__ void __launch_bounds__(kNetThreads) head_kernel(HeadArgs a) {
  __shared__ cplx<float> tab[kClasses * kStencilPts];
  __shared__ double red[kNetThreads / kWave];
  __shared__ float hw[C * 2 + 2];
  __shared__ float pred[kNetThreads / kWave][C * 2 + 2];
  const int b = blockIdx.x, tid = threadIdx.x, T = a.T, npix = T * T;
  for (int i = tid; i < 2 * C + 2; i += kNetThreads)
    hw[i] = i < 2 * C ? a.params[a.woff + i] : a.params[a.boff + i - 2 * C];
  TileDescDev d{0, 0, 0, 0, 0.0};
  if (a.t) {
    d = a.desc[b];
    build_class_table<float>(d.robin, d.kh, d.kh * d.kh, tab);
  }
  __syncthreads();
  const bf16* act = a.a7 + (size_t)b * npix * C;
  float* y = a.y + (size_t)b * npix * 2;
  const float* t = a.t ? a.t + (size_t)b * npix * 2 : nullptr;
  float* E = a.E ? a.E + (size_t)b * npix * 2 : nullptr;
  float* R = a.R ? a.R + (size_t)b * npix * 2 : nullptr;
  double num_err = 0.0, den_err = 0.0;
  for (int p = tid; p < npix; p += kNetThreads) {
    float y0 = hw[2 * C], y1 = hw[2 * C + 1];
    for (int c = 0; c < C; ++c) {
      const float v = (float)act[(size_t)p * C + c];
      y0 = fmaf(v, hw[2 * c], y0);
      y1 = fmaf(v, hw[2 * c + 1], y1);
    }
    y[2 * p] = y0;
    y[2 * p + 1] = y1;
    if (t) {
      const int li = p % T, lj = p / T;
      const bool node = li < d.nx && lj < d.ny;
      const float e0 = node ? y0 - t[2 * p] : 0.0f, e1 = node ? y1 - t[2 * p + 1] : 0.0f;
      E[2 * p] = e0;
      E[2 * p + 1] = e1;
      num_err += (double)e0 * e0 + (double)e1 * e1;
      if (node) den_err += (double)t[2 * p] * t[2 * p] + (double)t[2 * p + 1] * t[2 * p + 1];
    }
  }
  if (!t) return;
  __syncthreads();
  double num_res = 0.0, den_res = 0.0;
  auto getE = [&](int i, int j) { return cplx<float>{E[2 * (j * T + i)], E[2 * (j * T + i) + 1]}; };
  auto getT = [&](int i, int j) { return cplx<float>{t[2 * (j * T + i)], t[2 * (j * T + i) + 1]}; };
  for (int p = tid; p < npix; p += kNetThreads) {
    const int li = p % T, lj = p / T;
    cplx<float> r = czero<float>();
    if (li < d.nx && lj < d.ny) {
      r = tile_apply(tab, d, li, lj, getE);
      const cplx<float> bt = tile_apply(tab, d, li, lj, getT);
      num_res += (double)cabs2(r);
      den_res += (double)cabs2(bt);
    }
    R[2 * p] = r.re;
    R[2 * p + 1] = r.im;
  }
  num_err = block_sum_d(num_err, red);
  den_err = block_sum_d(den_err, red);
  num_res = block_sum_d(num_res, red);
  den_res = block_sum_d(den_res, red);
  if (den_err <= 0.0) den_err = 1.0;
  if (den_res <= 0.0) den_res = 1.0;
  if (tid == 0) a.loss[b] = a.w_res * num_res / den_res + a.w_err * num_err / den_err;
  const float sres = (float)(2.0 * a.w_res / (den_res * a.batch));
  const float serr = (float)(2.0 * a.w_err / (den_err * a.batch));
  // B^H r = conj(B conj(r)) (B is complex symmetric)
  auto getRc = [&](int i, int j) { return cplx<float>{R[2 * (j * T + i)], -R[2 * (j * T + i) + 1]}; };
  float pw[C * 2 + 2];
#pragma unroll
  for (int i = 0; i < 2 * C + 2; ++i) pw[i] = 0.0f;
  bf16* dz = a.dz7 + (size_t)b * npix * C;
  for (int p = tid; p < npix; p += kNetThreads) {
    const int li = p % T, lj = p / T;
    float g0 = 0.0f, g1 = 0.0f;
    if (li < d.nx && lj < d.ny) {
      const cplx<float> q = tile_apply(tab, d, li, lj, getRc);
      g0 = sres * q.re + serr * E[2 * p];
      g1 = -sres * q.im + serr * E[2 * p + 1];
    }
    pw[2 * C] += g0;
    pw[2 * C + 1] += g1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float v = (float)act[(size_t)p * C + c];
      pw[2 * c] = fmaf(v, g0, pw[2 * c]);
      pw[2 * c + 1] = fmaf(v, g1, pw[2 * c + 1]);
      const float da = g0 * hw[2 * c] + g1 * hw[2 * c + 1];
      dz[(size_t)p * C + c] = v > 0.0f ? (bf16)da : (bf16)0.0f;
    }
  }
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int i = 0; i < 2 * C + 2; ++i) {
    const float s = wave_sum(pw[i]);
    if (lane == 0) pred[wave][i] = s;
  }
  __syncthreads();
  for (int i = tid; i < 2 * C + 2; i += kNetThreads) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < kNetThreads / kWave; ++w) s += pred[w][i];
    if (i < 2 * C) a.part[(size_t)b * 2 * C + i] = s;
    else a.bpart[(size_t)b * 2 + i - 2 * C] = s;
  }
}

hipError_t launch_head(const HeadArgs& a, hipStream_t st) {
  switch (a.c1) {
    case 16: hipLaunchKernelGGL(head_kernel<16>, dim3(a.batch), dim3(kNetThreads), 0, st, a); break;
    case 32: hipLaunchKernelGGL(head_kernel<32>, dim3(a.batch), dim3(kNetThreads), 0, st, a); break;
    case 48: hipLaunchKernelGGL(head_kernel<48>, dim3(a.batch), dim3(kNetThreads), 0, st, a); break;
    case 64: hipLaunchKernelGGL(head_kernel<64>, dim3(a.batch), dim3(kNetThreads), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- optimiser -----------------------------------------------------------------------

// Adam (Kingma and Ba, 2015); c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st) {
  const int blocks = (int)std::min<long long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

// ---- tiles ---------------------------------------------------------------------------

__global__ void input_convert_kernel(const float* __restrict__ xf, bf16* __restrict__ xb, long long pixels) {
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < pixels;
       p += (long long)gridDim.x * blockDim.x) {
    const f32x4 v = *(const f32x4*)(xf + 4 * p);
    bf16x8 o = zero8();
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = (bf16)v[i];
    *(bf16x8*)(xb + 8 * p) = o;
  }
}

hipError_t launch_input_convert(const float* xf, bf16* xb, long long pixels, hipStream_t st) {
  const int blocks = (int)std::min<long long>((pixels + 255) / 256, 8192);
  hipLaunchKernelGGL(input_convert_kernel, dim3(blocks), dim3(256), 0, st, xf, xb, pixels);
  return hipGetLastError();
}

// Network input of solve (rhs, sub) = tile rhs * nsub + sub, from f = R_j r.
__global__ void __launch_bounds__(kNetThreads) tiles_kernel(TileArgs a) {
  __shared__ double red[kNetThreads / kWave];
  const int nsub = a.cs.nsub;
  const int b = blockIdx.x, rhs = b / nsub, sub = b - rhs * nsub;
  if (a.done && a.done[rhs]) return;
  const SubDesc d = a.subs[sub];
  const int T = a.T, nx = d.nx, nj = d.nx * d.ny, ldg = a.cs.n - 1;
  const long long jstep = a.jdev ? (long long)*a.jdev : 0;
  const cplx<double>* r = a.r + jstep * a.rslot + (long long)rhs * a.rstride;
  double s2 = 0.0;
  for (int n = threadIdx.x; n < nj; n += kNetThreads) {
    const int lj = n / nx, li = n - lj * nx;
    s2 += cabs2(r[(long long)(d.j0 + lj - 1) * ldg + (d.i0 + li - 1)]);
  }
  s2 = block_sum_d(s2, red);
  const double fn = sqrt(s2);
  const double s = fn > 0.0 ? sqrt((double)nj) / fn : 0.0;
  if (threadIdx.x == 0) a.scale[b] = s;
  const float kh = (float)a.cs.kh;
  for (int p = threadIdx.x; p < T * T; p += kNetThreads) {
    const int li = p % T, lj = p / T;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (li < d.nx && lj < d.ny) {
      const cplx<double> f = r[(long long)(d.j0 + lj - 1) * ldg + (d.i0 + li - 1)];
      const int cls = node_class(d.i0 + li, d.j0 + lj, d.ax, d.bx, d.ay, d.by);
      const int xc = cls % 3, yc = cls / 3;
      const bool imp = (xc == 0 && (d.robin & 1)) || (xc == 2 && (d.robin & 2)) || (yc == 0 && (d.robin & 4)) ||
                       (yc == 2 && (d.robin & 8));
      v[0] = (float)(s * f.re);
      v[1] = (float)(s * f.im);
      v[2] = kh;
      v[3] = imp ? -1.0f : 1.0f;
    }
    const size_t q = (size_t)b * T * T + p;
    if (a.xb) {
      bf16x8 o = zero8();
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = (bf16)v[i];
      *(bf16x8*)(a.xb + 8 * q) = o;
    }
    if (a.xf) *(f32x4*)(a.xf + 4 * q) = f32x4{v[0], v[1], v[2], v[3]};
  }
}

hipError_t launch_tiles(const TileArgs& a, int nsub, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(tiles_kernel, dim3(nsub * nrhs), dim3(kNetThreads), 0, st, a);
  return hipGetLastError();
}

// t[b][lj][li] = scale[b] * u[rhs][off + lj nx + li] on nodes, 0 elsewhere.
__global__ void packed_to_tiles_kernel(const SubDesc* __restrict__ subs, int nsub, long long nfine,
                                       const cplx<double>* __restrict__ u, const double* __restrict__ scale, int T,
                                       float* __restrict__ t) {
  const int b = blockIdx.x, rhs = b / nsub, sub = b - rhs * nsub;
  const SubDesc d = subs[sub];
  const double s = scale[b];
  for (int p = threadIdx.x; p < T * T; p += blockDim.x) {
    const int li = p % T, lj = p / T;
    float v0 = 0.f, v1 = 0.f;
    if (li < d.nx && lj < d.ny) {
      const cplx<double> x = u[(long long)rhs * nfine + d.off + (long long)lj * d.nx + li];
      v0 = (float)(s * x.re);
      v1 = (float)(s * x.im);
    }
    t[((size_t)b * T * T + p) * 2] = v0;
    t[((size_t)b * T * T + p) * 2 + 1] = v1;
  }
}

hipError_t launch_packed_to_tiles(const SubDesc* subs, int nsub, int nrhs, long long nfine,
                                  const cplx<double>* u, const double* scale, int T, float* t, hipStream_t st) {
  hipLaunchKernelGGL(packed_to_tiles_kernel, dim3(nsub * nrhs), dim3(256), 0, st, subs, nsub, nfine, u, scale, T, t);
  return hipGetLastError();
}

hipError_t configure_net() {
  const int lim = 160 * 1024;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)conv3x3_kernel<1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)conv3x3_kernel<2, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)conv3x3_kernel<4, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)conv3x3_kernel<8, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)conv3x3_kernel<1, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)conv3x3_kernel<2, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)conv3x3_kernel<4, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim)))
    return e;
  return hipFuncSetAttribute((const void*)conv3x3_wgrad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

}  // namespace ddh
