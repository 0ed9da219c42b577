// Learned preconditioner: a 3-level 3D convolutional U-Net (16/32/64 channels,
// 3x3x3 kernels, periodic padding) that corrects the homogeneous-reference
// preconditioner of the PCG (Sec. 3.3 eqs. matrixP, precond):
//     z = P^ r + F[ s e^{i phi} N_theta(x) ],
// x = [ e^{-i phi} F^-1(P^ r) / s  (6 real channels),  21 stiffness channels,
//       density ] in real space (s = RMS of F^-1(P^ r), phi its canonical phase).
// The network is nonlinear, so it runs inside flexible CG (Polak-Ribiere beta)
// with the plain preconditioner as fallback when a direction stops descending.
//
// Convolutions run on BF16 MFMA (v_mfma_f32_16x16x16bf16, FP32 accumulation) as
// implicit GEMMs over (voxels x output channels x 27 taps * input channels);
// activations are stored FP32 channels-last [sample][voxel][channel] and
// rounded to BF16 when fed to the matrix cores.  The weight gradient is an FP32
// reduction over voxels (deterministic two-phase sum).  Training minimizes the
// mean squared error between the network output and the normalized correction
// e^{-i phi} F^-1(x* - P^ r) / s for pairs (r, x* = K^-1 r) from plain PCG.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bw_block.h"
#include "bw_ops_impl.h"

namespace bw {

typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (short)(u >> 16);
}
static short f2bf_host(float x) {
  unsigned u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// ---------------------------------------------------------------------------
// architecture
// ---------------------------------------------------------------------------
struct LayerSpec {
  int cin, cout, taps;
};
constexpr int NLAYER = 9;
constexpr LayerSpec LAYERS[NLAYER] = {
    {32, 16, 27},  // 0: input (28 used) -> 16
    {16, 16, 27},  // 1
    {16, 32, 27},  // 2: after pool
    {32, 32, 27},  // 3
    {32, 64, 27},  // 4: after pool
    {64, 64, 27},  // 5
    {96, 32, 27},  // 6: upsample(64) ++ skip(32)
    {48, 16, 27},  // 7: upsample(32) ++ skip(16)
    {16, 16, 1},   // 8: 1x1x1 head, outputs 0..5 used
};
constexpr int NIN = 28, NOUT = 6;

static long layer_wcount(int l) { return (long)LAYERS[l].taps * LAYERS[l].cout * LAYERS[l].cin; }

}  // namespace bw

struct bw_unet {
  std::vector<float> w_host;      // flat: per layer W [taps][cout][cin] then bias [cout]
  std::vector<long> w_off, b_off;
  long nparam = 0;
  float* d_w = nullptr;           // FP32 master weights
  float* d_g = nullptr;           // gradient
  float* d_m = nullptr;           // Adam moments
  float* d_v = nullptr;
  short* d_wb = nullptr;          // BF16 copies [taps][cout][cin]
  short* d_wbt = nullptr;         // BF16 transposed + mirrored [taps][cin][cout]
  long adam_t = 0;
  int device = 0;
  bw::DevBuf act, grad, feat, tmp, part, vecs, qbuf, small;
};

namespace bw {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
struct Dims {
  int n0, n1, n2;
  long V;
};

__device__ __forceinline__ long nbr(const Dims& d, long v, int t) {
  const int i2 = (int)(v % d.n2);
  const long r = v / d.n2;
  const int i1 = (int)(r % d.n1), i0 = (int)(r / d.n1);
  const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  int j0 = i0 + dz, j1 = i1 + dy, j2 = i2 + dx;
  j0 += (j0 < 0) ? d.n0 : (j0 >= d.n0 ? -d.n0 : 0);
  j1 += (j1 < 0) ? d.n1 : (j1 >= d.n1 ? -d.n1 : 0);
  j2 += (j2 < 0) ? d.n2 : (j2 >= d.n2 ? -d.n2 : 0);
  return ((long)j0 * d.n1 + j1) * d.n2 + j2;
}

// Y[b][v][yoff + co] = act(bias[co] + sum_t sum_ci W[t][co][ci] X[b][nbr(v, t)][ci])
// (TAPS = 1: no neighbour).  One workgroup: 64 voxels x all COUT; wave w owns
// voxels 16 w .. 16 w + 15.  MFMA A = X tile (voxel x ci), B = W (ci x co).
template <int CIN, int COUT, int TAPS>
__global__ __launch_bounds__(256) void k_conv(const float* __restrict__ X, const short* __restrict__ Wb,
                                              const float* __restrict__ bias, float* __restrict__ Y, Dims d,
                                              int ystride, int yoff, int relu) {
  constexpr int NB = COUT / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long tiles = (d.V + 63) / 64;
  const int b = (int)(blockIdx.x / tiles);
  const long v0 = (blockIdx.x - (long)b * tiles) * 64 + wave * 16;
  const float* Xb = X + (size_t)b * d.V * CIN;
  const int i = lane & 15, kq = lane >> 4;
  const long v = v0 + i < d.V ? v0 + i : d.V - 1;  // partial tiles on tiny grids: clamp loads
  f4_t acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = f4_t{0, 0, 0, 0};
  for (int t = 0; t < TAPS; ++t) {
    const long nv = TAPS == 1 ? v : nbr(d, v, t);
    const float* xr = Xb + (size_t)nv * CIN;
#pragma unroll
    for (int c0 = 0; c0 < CIN; c0 += 16) {
      const float4 xv = *reinterpret_cast<const float4*>(xr + c0 + 4 * kq);
      bf4_t a;
      a[0] = f2bf(xv.x);
      a[1] = f2bf(xv.y);
      a[2] = f2bf(xv.z);
      a[3] = f2bf(xv.w);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const short* wr = Wb + ((size_t)(t * COUT + j * 16 + i) * CIN + c0 + 4 * kq);
        const bf4_t bb = *reinterpret_cast<const bf4_t*>(wr);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[j], 0, 0, 0);
      }
    }
  }
  float* Yb = Y + (size_t)b * d.V * ystride;
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long vo = v0 + 4 * kq + r;
      if (vo >= d.V) continue;
      const int co = j * 16 + i;
      float y = acc[j][r] + (bias ? bias[co] : 0.f);
      if (relu) y = y > 0.f ? y : 0.f;
      Yb[(size_t)vo * ystride + yoff + co] = y;
    }
}

// dW[t][co][ci] partial over a voxel chunk: sum_v dZ[v][co] X[nbr(v,t)][ci]
// (FP32); also db[co] partial (t == 0 blocks).  grid = (chunks, taps, B)
template <int CIN, int COUT, int TAPS>
__global__ __launch_bounds__(256) void k_conv_dw(const float* __restrict__ X, const float* __restrict__ dZ,
                                                 int dzstride, int dzoff, Dims d, long chunk,
                                                 float* __restrict__ part) {
  __shared__ float xs[32][CIN + 1];
  __shared__ float zs[32][COUT + 1];
  constexpr int NP = (CIN * COUT + 255) / 256;
  const int t = blockIdx.y, bb = blockIdx.z;
  const long vstart = (long)blockIdx.x * chunk;
  const long vend = vstart + chunk < d.V ? vstart + chunk : d.V;
  const float* Xb = X + (size_t)bb * d.V * CIN;
  const float* Zb = dZ + (size_t)bb * d.V * dzstride;
  float acc[NP], accb = 0.f;
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = 0.f;
  for (long v0 = vstart; v0 < vend; v0 += 32) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < 32 * CIN; idx += 256) {
      const int vv = idx / CIN, c = idx - vv * CIN;
      const long v = v0 + vv;
      xs[vv][c] = v < vend ? Xb[(size_t)(TAPS == 1 ? v : nbr(d, v, t)) * CIN + c] : 0.f;
    }
    for (int idx = threadIdx.x; idx < 32 * COUT; idx += 256) {
      const int vv = idx / COUT, c = idx - vv * COUT;
      const long v = v0 + vv;
      zs[vv][c] = v < vend ? Zb[(size_t)v * dzstride + dzoff + c] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int pair = threadIdx.x + p * 256;
      if (pair < CIN * COUT) {
        const int co = pair / CIN, ci = pair - co * CIN;
        float s = 0.f;
#pragma unroll 8
        for (int vv = 0; vv < 32; ++vv) s += zs[vv][co] * xs[vv][ci];
        acc[p] += s;
      }
    }
    if (t == 0 && threadIdx.x < COUT) {
      float s = 0.f;
      for (int vv = 0; vv < 32; ++vv) s += zs[vv][threadIdx.x];
      accb += s;
    }
  }
  // partial layout: [B][chunks][taps * COUT * CIN + COUT]
  const long per = (long)TAPS * COUT * CIN + COUT;
  float* pp = part + ((size_t)bb * gridDim.x + blockIdx.x) * per;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int pair = threadIdx.x + p * 256;
    if (pair < CIN * COUT) pp[(size_t)t * COUT * CIN + pair] = acc[p];
  }
  if (t == 0 && threadIdx.x < COUT) pp[(long)TAPS * COUT * CIN + threadIdx.x] = accb;
}

// sum the partials (fixed order) into the layer's gradient slice
__global__ void k_dw_reduce(const float* __restrict__ part, long per, int nparts, float* __restrict__ g) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < per; e += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int p = 0; p < nparts; ++p) s += part[(size_t)p * per + e];
    g[e] = s;
  }
}

// 2x2x2 average pooling, channels-last
__global__ void k_pool(const float* __restrict__ X, float* __restrict__ Y, Dims din, int C, int nb) {
  const int m0 = din.n0 / 2, m1 = din.n1 / 2, m2 = din.n2 / 2;
  const long Vo = (long)m0 * m1 * m2;
  const long total = (long)nb * Vo * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long vo = (e / C) % Vo;
    const int b = (int)(e / (C * Vo));
    const int j2 = (int)(vo % m2), j1 = (int)((vo / m2) % m1), j0 = (int)(vo / ((long)m1 * m2));
    float s = 0.f;
    for (int a = 0; a < 8; ++a) {
      const long vi = ((long)(2 * j0 + (a >> 2)) * din.n1 + 2 * j1 + ((a >> 1) & 1)) * din.n2 + 2 * j2 + (a & 1);
      s += X[((size_t)b * din.V + vi) * C + c];
    }
    Y[e] = 0.125f * s;
  }
}

// adjoint of the pooling: dX[fine] += dY[coarse] / 8 (written, not accumulated)
__global__ void k_pool_back(const float* __restrict__ dY, float* __restrict__ dX, Dims din, int C, int nb,
                            int dxstride, int dxoff, int accumulate) {
  const int m1 = din.n1 / 2, m2 = din.n2 / 2;
  const long Vo = (long)(din.n0 / 2) * m1 * m2;
  const long total = (long)nb * din.V * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long vi = (e / C) % din.V;
    const int b = (int)(e / (C * din.V));
    const int i2 = (int)(vi % din.n2), i1 = (int)((vi / din.n2) % din.n1), i0 = (int)(vi / ((long)din.n1 * din.n2));
    const long vo = ((long)(i0 / 2) * m1 + i1 / 2) * m2 + i2 / 2;
    const float g = 0.125f * dY[((size_t)b * Vo + vo) * C + c];
    float* dst = dX + ((size_t)b * din.V + vi) * dxstride + dxoff + c;
    *dst = accumulate ? *dst + g : g;
  }
}

// nearest upsampling (x2) of X [coarse][C] into Y[fine][0..C) of a buffer with ystride channels
__global__ void k_upsample(const float* __restrict__ X, float* __restrict__ Y, Dims dout, int C, int ystride,
                           int nb) {
  const int m1 = dout.n1 / 2, m2 = dout.n2 / 2;
  const long Vc = (long)(dout.n0 / 2) * m1 * m2;
  const long total = (long)nb * dout.V * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long vi = (e / C) % dout.V;
    const int b = (int)(e / (C * dout.V));
    const int i2 = (int)(vi % dout.n2), i1 = (int)((vi / dout.n2) % dout.n1), i0 = (int)(vi / ((long)dout.n1 * dout.n2));
    const long vc = ((long)(i0 / 2) * m1 + i1 / 2) * m2 + i2 / 2;
    Y[((size_t)b * dout.V + vi) * ystride + c] = X[((size_t)b * Vc + vc) * C + c];
  }
}

// adjoint of the upsampling: dX[coarse][c] = sum of the 8 fine dY[fine][c]
__global__ void k_upsample_back(const float* __restrict__ dY, int dystride, float* __restrict__ dX, Dims dout,
                                int C, int nb) {
  const int m0 = dout.n0 / 2, m1 = dout.n1 / 2, m2 = dout.n2 / 2;
  const long Vc = (long)m0 * m1 * m2;
  const long total = (long)nb * Vc * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long vc = (e / C) % Vc;
    const int b = (int)(e / (C * Vc));
    const int j2 = (int)(vc % m2), j1 = (int)((vc / m2) % m1), j0 = (int)(vc / ((long)m1 * m2));
    float s = 0.f;
    for (int a = 0; a < 8; ++a) {
      const long vi = ((long)(2 * j0 + (a >> 2)) * dout.n1 + 2 * j1 + ((a >> 1) & 1)) * dout.n2 + 2 * j2 + (a & 1);
      s += dY[((size_t)b * dout.V + vi) * dystride + c];
    }
    dX[e] = s;
  }
}

// copy C channels between channels-last buffers (concatenation)
__global__ void k_copy_ch(const float* __restrict__ X, int xstride, int xoff, float* __restrict__ Y, int ystride,
                          int yoff, long nvox, int C) {
  const long total = nvox * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long v = e / C;
    Y[(size_t)v * ystride + yoff + c] = X[(size_t)v * xstride + xoff + c];
  }
}

// dZ = dY * [Y > 0] (in place on dY with its stride), for nvox rows of C channels
__global__ void k_relu_back(float* __restrict__ dY, int stride, int off, const float* __restrict__ Y, int ystride,
                            int yoff, long nvox, int C) {
  const long total = nvox * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long v = e / C;
    if (Y[(size_t)v * ystride + yoff + c] <= 0.f) dY[(size_t)v * stride + off + c] = 0.f;
  }
}

// BF16 weight copies: W [taps][cout][cin] -> Wb (same layout) and Wbt [taps'][cin][cout]
// with the mirrored tap (27 - 1 - t) for the input-gradient convolution.
__global__ void k_wcast(const float* __restrict__ W, short* __restrict__ Wb, short* __restrict__ Wbt, int taps,
                        int cout, int cin) {
  const long n = (long)taps * cout * cin;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int ci = (int)(e % cin);
    const int co = (int)((e / cin) % cout);
    const int t = (int)(e / ((long)cin * cout));
    const short h = f2bf(W[e]);
    Wb[e] = h;
    const int tm = taps == 1 ? 0 : taps - 1 - t;
    Wbt[((size_t)tm * cin + ci) * cout + co] = h;
  }
}

// Adam step on the flat parameter vector; `frozen` entries (padded outputs /
// inputs) are kept at zero.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
  }
}

// squared error and its gradient of the head output (channels 0..5 of 16)
__global__ void k_mse(const float* __restrict__ out, const float* __restrict__ tgt, float* __restrict__ dout,
                      long nvox, float scale, double* __restrict__ partial) {
  __shared__ double sh[NT / 64];
  double s = 0;
  for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float dlt = 0.f;
      if (c < NOUT) {
        dlt = out[(size_t)v * 16 + c] - tgt[(size_t)v * NOUT + c];
        s += (double)dlt * dlt;
      }
      dout[(size_t)v * 16 + c] = 2.f * scale * dlt;
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Bloch-field <-> network channels
// ---------------------------------------------------------------------------
// sum over voxels and components of e_c(v)^2 (complex) and of |e_c(v)|^2, per sample
__global__ void k_phase_stats(const float2* __restrict__ E, long nvox, int bpv, double* __restrict__ partial) {
  __shared__ double sh[NT / 64];
  const int b = blockIdx.x / bpv, blk = blockIdx.x - b * bpv;
  double sr = 0, si = 0, ss = 0;
  for (long v = (long)blk * NT + threadIdx.x; v < nvox; v += (long)bpv * NT)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float2 e = E[((size_t)b * 3 + c) * nvox + v];
      sr += (double)e.x * e.x - (double)e.y * e.y;
      si += 2.0 * (double)e.x * e.y;
      ss += (double)e.x * e.x + (double)e.y * e.y;
    }
  const double vals[3] = {sr, si, ss};
  store_partials<3>(vals, partial, b, blk, bpv, sh);
}

// x[b][v][0..5] = e^{-i phi_b} E_c(v) / s_b ; x[b][v][6..31] = static material channels
__global__ void k_features(const float2* __restrict__ E, const float* __restrict__ mat, const double* __restrict__ ps,
                           float* __restrict__ x, long nvox, int nb) {
  const long total = (long)nb * nvox;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long v = e % nvox;
    const int b = (int)(e / nvox);
    const float cr = (float)ps[4 * b], ci = (float)ps[4 * b + 1], is = (float)ps[4 * b + 2];
    float* xr = x + (size_t)e * 32;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float2 z = E[((size_t)b * 3 + c) * nvox + v];
      // (z.x + i z.y)(cr - i ci) / s   with (cr, ci) = e^{i phi}
      xr[2 * c] = (z.x * cr + z.y * ci) * is;
      xr[2 * c + 1] = (z.y * cr - z.x * ci) * is;
    }
    const float* m = mat + (size_t)v * 26;
#pragma unroll
    for (int c = 0; c < 26; ++c) xr[6 + c] = m[c];
  }
}

// target t[b][v][c] = e^{-i phi} D_c(v) / s (D = F^-1(x* - P^ r) in real space)
__global__ void k_target(const float2* __restrict__ D, const double* __restrict__ ps, float* __restrict__ t, long nvox,
                         int nb) {
  const long total = (long)nb * nvox;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long v = e % nvox;
    const int b = (int)(e / nvox);
    const float cr = (float)ps[4 * b], ci = (float)ps[4 * b + 1], is = (float)ps[4 * b + 2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float2 z = D[((size_t)b * 3 + c) * nvox + v];
      t[(size_t)e * NOUT + 2 * c] = (z.x * cr + z.y * ci) * is;
      t[(size_t)e * NOUT + 2 * c + 1] = (z.y * cr - z.x * ci) * is;
    }
  }
}

// gradient of the residual loss with respect to the head output: with h = F^H g
// (g the gradient with respect to conj z, already divided by ||r||^2), the output
// o_{2c} + i o_{2c+1} enters z through F[s e^{i phi} (.)], so
// dL/do_{2c} = fac s Re(e^{-i phi} h_c), dL/do_{2c+1} = fac s Im(e^{-i phi} h_c).
__global__ void k_outgrad(const float2* __restrict__ H, const double* __restrict__ ps, float* __restrict__ dout,
                          long nvox, int nb, float fac) {
  const long total = (long)nb * nvox;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long v = e % nvox;
    const int b = (int)(e / nvox);
    const float cr = (float)ps[4 * b], ci = (float)ps[4 * b + 1], f = fac * (float)ps[4 * b + 3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float2 h = H[((size_t)b * 3 + c) * nvox + v];
      dout[(size_t)e * 16 + 2 * c] = f * (h.x * cr + h.y * ci);
      dout[(size_t)e * 16 + 2 * c + 1] = f * (h.y * cr - h.x * ci);
    }
#pragma unroll
    for (int c = 6; c < 16; ++c) dout[(size_t)e * 16 + c] = 0.f;
  }
}

// network output -> real-space correction D_c(v) = s e^{i phi} (o_{2c} + i o_{2c+1})
__global__ void k_output(const float* __restrict__ o, const double* __restrict__ ps, float2* __restrict__ D,
                         long nvox, int nb) {
  const long total = (long)nb * nvox;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long v = e % nvox;
    const int b = (int)(e / nvox);
    const float cr = (float)ps[4 * b], ci = (float)ps[4 * b + 1], s = (float)ps[4 * b + 3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float a = o[(size_t)e * 16 + 2 * c], bb = o[(size_t)e * 16 + 2 * c + 1];
      D[((size_t)b * 3 + c) * nvox + v] = make_float2(s * (a * cr - bb * ci), s * (a * ci + bb * cr));
    }
  }
}

// static material channels per voxel: 21 scaled stiffness entries, scaled density, 4 zeros
__global__ void k_material(const uint16_t* __restrict__ gmap, const float* __restrict__ C, const float* __restrict__ rho,
                           float* __restrict__ mat, long nvox) {
  for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long)gridDim.x * blockDim.x) {
    const int g = gmap[v];
#pragma unroll
    for (int c = 0; c < 21; ++c) mat[(size_t)v * 26 + c] = C[g * 21 + c];
    mat[(size_t)v * 26 + 21] = rho[g];
#pragma unroll
    for (int c = 22; c < 26; ++c) mat[(size_t)v * 26 + c] = 0.f;
  }
}

}  // namespace bw

namespace bw {

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------
static Dims dims_of(int n0, int n1, int n2) { return Dims{n0, n1, n2, (long)n0 * n1 * n2}; }
static unsigned grid_for(long n) {
  long b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

template <int CIN, int COUT, int TAPS>
static void conv(const float* X, const short* W, const float* bias, float* Y, Dims d, int nb, int ystride, int yoff,
                 bool relu, hipStream_t s) {
  const long tiles = (d.V + 63) / 64;
  BW_LAUNCH("k_conv_bf16_mfma", (long)nb * d.V, (k_conv<CIN, COUT, TAPS>), dim3((unsigned)(nb * tiles)), dim3(256),
            0, s, X, W, bias, Y, d, ystride, yoff, relu ? 1 : 0);
}

template <int CIN, int COUT, int TAPS>
static void conv_dw(const float* X, const float* dZ, int dzstride, int dzoff, Dims d, int nb, float* part,
                    float* g, hipStream_t s) {
  long chunks = (d.V + 4095) / 4096;
  if (chunks < 1) chunks = 1;
  const long chunk = (d.V + chunks - 1) / chunks;
  const long per = (long)TAPS * COUT * CIN + COUT;
  hipLaunchKernelGGL((k_conv_dw<CIN, COUT, TAPS>), dim3((unsigned)chunks, TAPS, nb), dim3(256), 0, s, X, dZ,
                     dzstride, dzoff, d, chunk, part);
  hipLaunchKernelGGL(k_dw_reduce, dim3(grid_for(per)), dim3(256), 0, s, (const float*)part, per,
                     (int)(nb * chunks), g);
}

struct Acts {  // activations (forward) and gradients (backward), channels-last FP32
  float *X0, *A1, *S1, *P1, *A2, *S2, *P2, *A3, *B3, *C2, *A4, *C1, *A5, *O;
  float *dO, *dC1, *dA4, *dC2, *dB3, *dA3, *dP2, *dS2, *dA2, *dP1, *dS1, *dA1, *dA5, *part;
};

static Acts acts_for(bw_unet* u, Dims d1, int nb, bool backward) {
  const long V1 = d1.V, V2 = V1 / 8, V3 = V1 / 64;
  const long fw = (long)nb * (V1 * (32 + 16 + 16 + 48 + 16 + 16) + V2 * (16 + 32 + 32 + 96 + 32) + V3 * (32 + 64 + 64));
  float* a = (float*)u->act.get((size_t)fw * sizeof(float));
  Acts t{};
  auto take = [&](long n) {
    float* p = a;
    a += n;
    return p;
  };
  t.X0 = take(nb * V1 * 32);
  t.A1 = take(nb * V1 * 16);
  t.S1 = take(nb * V1 * 16);
  t.C1 = take(nb * V1 * 48);
  t.A5 = take(nb * V1 * 16);
  t.O = take(nb * V1 * 16);
  t.P1 = take(nb * V2 * 16);
  t.A2 = take(nb * V2 * 32);
  t.S2 = take(nb * V2 * 32);
  t.C2 = take(nb * V2 * 96);
  t.A4 = take(nb * V2 * 32);
  t.P2 = take(nb * V3 * 32);
  t.A3 = take(nb * V3 * 64);
  t.B3 = take(nb * V3 * 64);
  if (backward) {
    const long bw = (long)nb * (V1 * (16 + 48 + 16 + 16 + 16) + V2 * (32 + 96 + 32 + 32 + 16) + V3 * (64 + 64 + 32));
    long maxper = 0;
    for (int l = 0; l < NLAYER; ++l) maxper = std::max(maxper, layer_wcount(l) + LAYERS[l].cout);
    const long chunks1 = (V1 + 4095) / 4096;
    float* g = (float*)u->grad.get((size_t)(bw + (long)nb * chunks1 * maxper) * sizeof(float));
    auto takeg = [&](long n) {
      float* p = g;
      g += n;
      return p;
    };
    t.dO = takeg(nb * V1 * 16);
    t.dC1 = takeg(nb * V1 * 48);
    t.dS1 = takeg(nb * V1 * 16);
    t.dA1 = takeg(nb * V1 * 16);
    t.dA5 = takeg(nb * V1 * 16);
    t.dA4 = takeg(nb * V2 * 32);
    t.dC2 = takeg(nb * V2 * 96);
    t.dS2 = takeg(nb * V2 * 32);
    t.dA2 = takeg(nb * V2 * 32);
    t.dP1 = takeg(nb * V2 * 16);
    t.dB3 = takeg(nb * V3 * 64);
    t.dA3 = takeg(nb * V3 * 64);
    t.dP2 = takeg(nb * V3 * 32);
    t.part = g;
  }
  return t;
}

static const short* WB(bw_unet* u, int l) { return u->d_wb + u->w_off[l]; }
static const short* WT(bw_unet* u, int l) { return u->d_wbt + u->w_off[l]; }
static const float* BI(bw_unet* u, int l) { return u->d_w + u->b_off[l]; }

static void unet_forward(bw_unet* u, Acts& a, Dims d1, int nb, hipStream_t s) {
  const Dims d2 = dims_of(d1.n0 / 2, d1.n1 / 2, d1.n2 / 2), d3 = dims_of(d1.n0 / 4, d1.n1 / 4, d1.n2 / 4);
  conv<32, 16, 27>(a.X0, WB(u, 0), BI(u, 0), a.A1, d1, nb, 16, 0, true, s);
  conv<16, 16, 27>(a.A1, WB(u, 1), BI(u, 1), a.S1, d1, nb, 16, 0, true, s);
  hipLaunchKernelGGL(k_pool, dim3(grid_for(nb * d2.V * 16)), dim3(256), 0, s, a.S1, a.P1, d1, 16, nb);
  conv<16, 32, 27>(a.P1, WB(u, 2), BI(u, 2), a.A2, d2, nb, 32, 0, true, s);
  conv<32, 32, 27>(a.A2, WB(u, 3), BI(u, 3), a.S2, d2, nb, 32, 0, true, s);
  hipLaunchKernelGGL(k_pool, dim3(grid_for(nb * d3.V * 32)), dim3(256), 0, s, a.S2, a.P2, d2, 32, nb);
  conv<32, 64, 27>(a.P2, WB(u, 4), BI(u, 4), a.A3, d3, nb, 64, 0, true, s);
  conv<64, 64, 27>(a.A3, WB(u, 5), BI(u, 5), a.B3, d3, nb, 64, 0, true, s);
  hipLaunchKernelGGL(k_upsample, dim3(grid_for(nb * d2.V * 64)), dim3(256), 0, s, a.B3, a.C2, d2, 64, 96, nb);
  hipLaunchKernelGGL(k_copy_ch, dim3(grid_for(nb * d2.V * 32)), dim3(256), 0, s, a.S2, 32, 0, a.C2, 96, 64,
                     (long)nb * d2.V, 32);
  conv<96, 32, 27>(a.C2, WB(u, 6), BI(u, 6), a.A4, d2, nb, 32, 0, true, s);
  hipLaunchKernelGGL(k_upsample, dim3(grid_for(nb * d1.V * 32)), dim3(256), 0, s, a.A4, a.C1, d1, 32, 48, nb);
  hipLaunchKernelGGL(k_copy_ch, dim3(grid_for(nb * d1.V * 16)), dim3(256), 0, s, a.S1, 16, 0, a.C1, 48, 32,
                     (long)nb * d1.V, 16);
  conv<48, 16, 27>(a.C1, WB(u, 7), BI(u, 7), a.A5, d1, nb, 16, 0, true, s);
  conv<16, 16, 1>(a.A5, WB(u, 8), BI(u, 8), a.O, d1, nb, 16, 0, false, s);
}

// backward from dO (already in a.dO); fills u->d_g
static void unet_backward(bw_unet* u, Acts& a, Dims d1, int nb, hipStream_t s) {
  const Dims d2 = dims_of(d1.n0 / 2, d1.n1 / 2, d1.n2 / 2), d3 = dims_of(d1.n0 / 4, d1.n1 / 4, d1.n2 / 4);
  float* G = u->d_g;
  auto gW = [&](int l) { return G + u->w_off[l]; };
  auto relub = [&](float* dY, const float* Y, long nvox, int C) {
    hipLaunchKernelGGL(k_relu_back, dim3(grid_for(nvox * C)), dim3(256), 0, s, dY, C, 0, Y, C, 0, nvox, C);
  };
  // layer 8 (head)
  conv_dw<16, 16, 1>(a.A5, a.dO, 16, 0, d1, nb, a.part, gW(8), s);
  conv<16, 16, 1>(a.dO, WT(u, 8), nullptr, a.dA5, d1, nb, 16, 0, false, s);
  relub(a.dA5, a.A5, nb * d1.V, 16);
  // layer 7
  conv_dw<48, 16, 27>(a.C1, a.dA5, 16, 0, d1, nb, a.part, gW(7), s);
  conv<16, 48, 27>(a.dA5, WT(u, 7), nullptr, a.dC1, d1, nb, 48, 0, false, s);
  hipLaunchKernelGGL(k_upsample_back, dim3(grid_for(nb * d2.V * 32)), dim3(256), 0, s, a.dC1, 48, a.dA4, d1, 32, nb);
  relub(a.dA4, a.A4, nb * d2.V, 32);
  // layer 6
  conv_dw<96, 32, 27>(a.C2, a.dA4, 32, 0, d2, nb, a.part, gW(6), s);
  conv<32, 96, 27>(a.dA4, WT(u, 6), nullptr, a.dC2, d2, nb, 96, 0, false, s);
  hipLaunchKernelGGL(k_upsample_back, dim3(grid_for(nb * d3.V * 64)), dim3(256), 0, s, a.dC2, 96, a.dB3, d2, 64, nb);
  relub(a.dB3, a.B3, nb * d3.V, 64);
  // layer 5
  conv_dw<64, 64, 27>(a.A3, a.dB3, 64, 0, d3, nb, a.part, gW(5), s);
  conv<64, 64, 27>(a.dB3, WT(u, 5), nullptr, a.dA3, d3, nb, 64, 0, false, s);
  relub(a.dA3, a.A3, nb * d3.V, 64);
  // layer 4
  conv_dw<32, 64, 27>(a.P2, a.dA3, 64, 0, d3, nb, a.part, gW(4), s);
  conv<64, 32, 27>(a.dA3, WT(u, 4), nullptr, a.dP2, d3, nb, 32, 0, false, s);
  // skip 2: dS2 = dC2[:, 64:96] + pool^T dP2
  hipLaunchKernelGGL(k_copy_ch, dim3(grid_for(nb * d2.V * 32)), dim3(256), 0, s, a.dC2, 96, 64, a.dS2, 32, 0,
                     (long)nb * d2.V, 32);
  hipLaunchKernelGGL(k_pool_back, dim3(grid_for(nb * d2.V * 32)), dim3(256), 0, s, a.dP2, a.dS2, d2, 32, nb, 32, 0, 1);
  relub(a.dS2, a.S2, nb * d2.V, 32);
  // layer 3
  conv_dw<32, 32, 27>(a.A2, a.dS2, 32, 0, d2, nb, a.part, gW(3), s);
  conv<32, 32, 27>(a.dS2, WT(u, 3), nullptr, a.dA2, d2, nb, 32, 0, false, s);
  relub(a.dA2, a.A2, nb * d2.V, 32);
  // layer 2
  conv_dw<16, 32, 27>(a.P1, a.dA2, 32, 0, d2, nb, a.part, gW(2), s);
  conv<32, 16, 27>(a.dA2, WT(u, 2), nullptr, a.dP1, d2, nb, 16, 0, false, s);
  // skip 1: dS1 = dC1[:, 32:48] + pool^T dP1
  hipLaunchKernelGGL(k_copy_ch, dim3(grid_for(nb * d1.V * 16)), dim3(256), 0, s, a.dC1, 48, 32, a.dS1, 16, 0,
                     (long)nb * d1.V, 16);
  hipLaunchKernelGGL(k_pool_back, dim3(grid_for(nb * d1.V * 16)), dim3(256), 0, s, a.dP1, a.dS1, d1, 16, nb, 16, 0, 1);
  relub(a.dS1, a.S1, nb * d1.V, 16);
  // layer 1
  conv_dw<16, 16, 27>(a.A1, a.dS1, 16, 0, d1, nb, a.part, gW(1), s);
  conv<16, 16, 27>(a.dS1, WT(u, 1), nullptr, a.dA1, d1, nb, 16, 0, false, s);
  relub(a.dA1, a.A1, nb * d1.V, 16);
  // layer 0 (no input gradient needed)
  conv_dw<32, 16, 27>(a.X0, a.dA1, 16, 0, d1, nb, a.part, gW(0), s);
}

static void refresh_bf16(bw_unet* u, hipStream_t s) {
  for (int l = 0; l < NLAYER; ++l) {
    const long n = layer_wcount(l);
    hipLaunchKernelGGL(k_wcast, dim3(grid_for(n)), dim3(256), 0, s, (const float*)(u->d_w + u->w_off[l]),
                       u->d_wb + u->w_off[l], u->d_wbt + u->w_off[l], LAYERS[l].taps, LAYERS[l].cout,
                       LAYERS[l].cin);
  }
}

// zero the weights that touch padded channels (inputs 28..31 of layer 0, outputs 6..15 of the head)
static void mask_padding(bw_unet* u) {
  for (int t = 0; t < 27; ++t)
    for (int co = 0; co < 16; ++co)
      for (int ci = NIN; ci < 32; ++ci) u->w_host[u->w_off[0] + ((long)t * 16 + co) * 32 + ci] = 0.f;
  for (int co = NOUT; co < 16; ++co) {
    for (int ci = 0; ci < 16; ++ci) u->w_host[u->w_off[8] + (long)co * 16 + ci] = 0.f;
    u->w_host[u->b_off[8] + co] = 0.f;
  }
}

static void upload_weights(bw_unet* u, hipStream_t s) {
  BW_HIP(hipMemcpy(u->d_w, u->w_host.data(), u->nparam * sizeof(float), hipMemcpyHostToDevice));
  refresh_bf16(u, s);
  BW_HIP(hipStreamSynchronize(s));
}

// gradient entries of padded channels are zeroed so Adam keeps them at zero
__global__ void k_mask_grad(float* g, long off0, long off8, long boff8) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 27 * 16 * 4) {
    const int tap = t / 64, co = (t / 4) % 16, ci = NIN + t % 4;
    g[off0 + ((long)tap * 16 + co) * 32 + ci] = 0.f;
  }
  if (t < 10 * 16) {
    const int co = NOUT + t / 16, ci = t % 16;
    g[off8 + (long)co * 16 + ci] = 0.f;
  }
  if (t < 10) g[boff8 + NOUT + t] = 0.f;
}

// ---------------------------------------------------------------------------
// Bloch fields <-> channels
// ---------------------------------------------------------------------------
// Unnormalized 3D inverse (INV) or forward transform of nv three-component fields, in place.
template <bool INV> static void fft3_inplace(const bw_rve* r, float2* X, int nv, hipStream_t s) {
  const Geom& g = r->g;
  const long rows = 3L * g.n0 * g.n1;
  with_n(g.n2, [&](auto N2) {
    constexpr int n2c = decltype(N2)::value;
    RowTile rt = row_tile<float>(n2c, rows);
    hipLaunchKernelGGL((k_row_plain<float, n2c, INV>), dim3(nv * rt.tpv), dim3(NT), 0, s, (const float2*)X, X, rt,
                       (int)rows, twiddles<float>(r, 2), (const int*)nullptr);
  });
  if (g.n1 > 1)
    with_n(g.n1, [&](auto N1) {
      ColTile ct = axis1_tile<float>(N1, g.n2, 3L * g.n0 * g.n2);
      hipLaunchKernelGGL((k_axis1<float, decltype(N1)::value, INV>), dim3(nv * ct.tpv), dim3(NT), 0, s, X, g.n2,
                         3L * g.nvox, ct, twiddles<float>(r, 1), (const int*)nullptr);
    });
  if (g.n0 > 1) {
    const int n12 = g.n1 * g.n2;
    with_n(g.n0, [&](auto N0) {
      ColTile ct = axis1_tile<float>(N0, n12, 3L * n12);
      hipLaunchKernelGGL((k_axis1<float, decltype(N0)::value, INV>), dim3(nv * ct.tpv), dim3(NT), 0, s, X, n12,
                         3L * g.nvox, ct, twiddles<float>(r, 0), (const int*)nullptr);
    });
  }
}

__global__ void k_finalize_phase(const double* partial, int bpv, long nvox, double* ps) {
  __shared__ double sh[NT / 64];
  double tot[3];
  sum_partials<3>(tot, partial, blockIdx.x, bpv, bpv, sh);
  if (threadIdx.x == 0) {
    const double ph = 0.5 * atan2(tot[1], tot[0]);
    const double rms = sqrt(tot[2] / (3.0 * (double)nvox));
    ps[4 * blockIdx.x] = cos(ph);
    ps[4 * blockIdx.x + 1] = sin(ph);
    ps[4 * blockIdx.x + 2] = rms > 0 ? 1.0 / rms : 0.0;
    ps[4 * blockIdx.x + 3] = rms / (double)nvox;  // output scale: s, and 1/N of the forward transform
  }
}

struct Feat {
  float2 *Z0, *E;
  float* mat;
  double* ps;
  double* part;
};

static Feat feat_bufs(bw_unet* u, const bw_rve* r, int nb) {
  const long n3 = r->g.nvox * 3;
  const int bpv = pw_blocks(r->g.nvox);
  char* p = (char*)u->feat.get((size_t)2 * nb * n3 * sizeof(float2) + (size_t)r->g.nvox * 26 * sizeof(float) +
                               (size_t)nb * 4 * sizeof(double) + (size_t)nb * bpv * 3 * sizeof(double) + 1024);
  Feat f;
  f.Z0 = (float2*)p;
  f.E = f.Z0 + (size_t)nb * n3;
  f.mat = (float*)(f.E + (size_t)nb * n3);
  f.ps = (double*)(f.mat + (size_t)r->g.nvox * 26);
  f.part = f.ps + (size_t)nb * 4;
  return f;
}

// features of nb residuals R (Fourier, FP32) into a.X0; Z0 = P^ R kept in f.Z0
static void build_features(const bw_rve* r, const double* dq, const float2* R, int nb, double pscale, Feat& f,
                           Acts& a, hipStream_t s) {
  const long nvox = r->g.nvox;
  launch_apply_P<float>(r, dq, R, f.Z0, nb, pscale, s);
  BW_HIP(hipMemcpyAsync(f.E, f.Z0, (size_t)nb * 3 * nvox * sizeof(float2), hipMemcpyDeviceToDevice, s));
  fft3_inplace<true>(r, f.E, nb, s);
  const int bpv = pw_blocks(nvox);
  hipLaunchKernelGGL(k_phase_stats, dim3(nb * bpv), dim3(NT), 0, s, (const float2*)f.E, nvox, bpv, f.part);
  hipLaunchKernelGGL(k_finalize_phase, dim3(nb), dim3(NT), 0, s, (const double*)f.part, bpv, nvox, f.ps);
  hipLaunchKernelGGL(k_material, dim3(grid_for(nvox)), dim3(256), 0, s, r->d_gmap, r->d_C32, r->d_rho32, f.mat, nvox);
  hipLaunchKernelGGL(k_features, dim3(grid_for(nb * nvox)), dim3(256), 0, s, (const float2*)f.E, (const float*)f.mat,
                     (const double*)f.ps, a.X0, nvox, nb);
}

__global__ void k_add_to(const float2* __restrict__ a, float2* __restrict__ y, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float2 u = a[e], w = y[e];
    y[e] = make_float2(u.x + w.x, u.y + w.y);
  }
}

// z = Z0 + F[output]  (into Zout)
static void apply_output(const bw_rve* r, Feat& f, Acts& a, float2* Zout, int nb, hipStream_t s) {
  const long nvox = r->g.nvox;
  hipLaunchKernelGGL(k_output, dim3(grid_for(nb * nvox)), dim3(256), 0, s, (const float*)a.O, (const double*)f.ps, Zout,
                     nvox, nb);
  fft3_inplace<false>(r, Zout, nb, s);
  hipLaunchKernelGGL(k_add_to, dim3(grid_for(nb * nvox * 3)), dim3(256), 0, s, (const float2*)f.Z0, Zout,
                     (long)nb * nvox * 3);
}

}  // namespace bw

namespace bw {

// ---------------------------------------------------------------------------
// parameters
// ---------------------------------------------------------------------------
static void init_layout(bw_unet* u) {
  long off = 0;
  u->w_off.assign(NLAYER, 0);
  u->b_off.assign(NLAYER, 0);
  for (int l = 0; l < NLAYER; ++l) {
    u->w_off[l] = off;
    off += layer_wcount(l);
    u->b_off[l] = off;
    off += LAYERS[l].cout;
  }
  u->nparam = off;
}

static uint64_t splitmix64(uint64_t& x) {
  x += 0x9E3779B97F4A7C15ull;
  uint64_t z = x;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double uniform01(uint64_t& st) { return ((double)(splitmix64(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

// He-normal weights (Box-Muller), zero biases, zero head: the untrained
// network adds nothing to the plain preconditioner.
static void he_init(bw_unet* u, uint64_t seed) {
  uint64_t st = seed * 0x2545F4914F6CDD1Dull + 2106124870ull;
  u->w_host.assign(u->nparam, 0.f);
  for (int l = 0; l + 1 < NLAYER; ++l) {
    const int cin_used = l == 0 ? NIN : LAYERS[l].cin;
    const double sd = std::sqrt(2.0 / ((double)LAYERS[l].taps * cin_used));
    for (long e = 0; e < layer_wcount(l); ++e) {
      const double a = uniform01(st), b = uniform01(st);
      u->w_host[u->w_off[l] + e] = (float)(sd * std::sqrt(-2.0 * std::log(a)) * std::cos(2.0 * M_PI * b));
    }
  }
  mask_padding(u);
}

static void check_grid(const int n[3]) {
  for (int a = 0; a < 3; ++a)
    BW_REQUIRE(n[a] >= 4 && n[a] % 4 == 0, BW_EUNSUPPORTED,
               "the learned preconditioner needs every grid size divisible by 4 (two 2x2x2 poolings)");
}

__global__ void k_fcg_update(float2* __restrict__ x, float2* __restrict__ r, const float2* __restrict__ p,
                             const float2* __restrict__ Kp, const double2* __restrict__ alpha, long n) {
  const int v = blockIdx.y;
  const double2 a = alpha[v];
  if (a.x == 0.0 && a.y == 0.0) return;
  const float ar = (float)a.x, ai = (float)a.y;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const size_t i = (size_t)v * n + e;
    const float2 pe = p[i], ke = Kp[i];
    float2 xe = x[i], re = r[i];
    xe.x += ar * pe.x - ai * pe.y;
    xe.y += ar * pe.y + ai * pe.x;
    re.x -= ar * ke.x - ai * ke.y;
    re.y -= ar * ke.y + ai * ke.x;
    x[i] = xe;
    r[i] = re;
  }
}

// p = z + beta p (beta complex, per vector); skip[v] leaves p untouched
__global__ void k_fcg_dir(float2* __restrict__ p, const float2* __restrict__ z, const double2* __restrict__ beta,
                          const int* __restrict__ skip, long n) {
  const int v = blockIdx.y;
  if (skip[v]) return;
  const float br = (float)beta[v].x, bi = (float)beta[v].y;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const size_t i = (size_t)v * n + e;
    const float2 pe = p[i], ze = z[i];
    p[i] = make_float2(ze.x + br * pe.x - bi * pe.y, ze.y + br * pe.y + bi * pe.x);
  }
}

// r = b - y
__global__ void k_sub(const float2* __restrict__ b, const float2* __restrict__ y, float2* __restrict__ r, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float2 u = b[e], w = y[e];
    r[e] = make_float2(u.x - w.x, u.y - w.y);
  }
}

static dim3 vec_grid(long n, int nv) {
  long b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  return dim3((unsigned)b, (unsigned)nv);
}

// Learned preconditioner on nb residuals (per-vector q tables in dq):
// Z = pscale P^ R + F[ s e^{i phi} N(x) ].  The null voxel (if any) is zeroed.
static void learned_apply(bw_unet* u, const bw_rve* r, const double* dq, const float2* R, float2* Z, int nb,
                          double pscale, const std::vector<int>& nullv, hipStream_t s) {
  const Geom& g = r->g;
  const Dims d1 = dims_of(g.n0, g.n1, g.n2);
  Acts a = acts_for(u, d1, nb, false);
  Feat f = feat_bufs(u, r, nb);
  build_features(r, dq, R, nb, pscale, f, a, s);
  unet_forward(u, a, d1, nb, s);
  apply_output(r, f, a, Z, nb, s);
  for (int v = 0; v < nb; ++v)
    if (nullv[v] >= 0) zero_voxel<float>(Z + (size_t)v * 3 * g.nvox, 1, g.nvox, nullv[v], s);
}

static std::vector<int> null_voxels(const QTable& qt) { return qt.null_index; }

}  // namespace bw

using namespace bw;

#define BWU_GUARD_BEGIN try {
#define BWU_GUARD_END                                      \
  }                                                        \
  catch (const bw::Error& e) {                             \
    bw::set_error(e.msg);                                  \
    return e.code;                                         \
  }                                                        \
  catch (const std::exception& e) {                        \
    bw::set_error(std::string("internal: ") + e.what());   \
    return BW_EINVAL;                                      \
  }

extern "C" int64_t bw_unet_param_count(void) {
  bw_unet tmp;
  init_layout(&tmp);
  return tmp.nparam;
}

extern "C" void bw_unet_destroy(bw_unet* u) {
  if (!u) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(u->device);
  (void)hipFree(u->d_w);
  (void)hipFree(u->d_g);
  (void)hipFree(u->d_m);
  (void)hipFree(u->d_v);
  (void)hipFree(u->d_wb);
  (void)hipFree(u->d_wbt);
  for (DevBuf* b : {&u->act, &u->grad, &u->feat, &u->tmp, &u->part, &u->vecs, &u->qbuf, &u->small}) b->release();
  (void)hipSetDevice(cur);
  delete u;
}

extern "C" int bw_unet_create(bw_unet** out, uint64_t seed) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(out, BW_EINVAL, "null argument");
  *out = nullptr;
  bw_unet* u = new bw_unet();
  try {
    BW_HIP(hipGetDevice(&u->device));
    init_layout(u);
    he_init(u, seed);
    const size_t nb4 = (size_t)u->nparam * sizeof(float);
    BW_HIP(hipMalloc(&u->d_w, nb4));
    BW_HIP(hipMalloc(&u->d_g, nb4));
    BW_HIP(hipMalloc(&u->d_m, nb4));
    BW_HIP(hipMalloc(&u->d_v, nb4));
    BW_HIP(hipMalloc(&u->d_wb, (size_t)u->nparam * sizeof(short)));
    BW_HIP(hipMalloc(&u->d_wbt, (size_t)u->nparam * sizeof(short)));
    BW_HIP(hipMemset(u->d_g, 0, nb4));
    BW_HIP(hipMemset(u->d_m, 0, nb4));
    BW_HIP(hipMemset(u->d_v, 0, nb4));
    upload_weights(u, nullptr);
  } catch (...) {
    bw_unet_destroy(u);
    throw;
  }
  *out = u;
  return BW_OK;
  BWU_GUARD_END
}

extern "C" int bw_unet_get_weights(const bw_unet* u, float* w_host, int64_t n) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(u && w_host, BW_EINVAL, "null argument");
  BW_REQUIRE(n == u->nparam, BW_EINVAL, "parameter count mismatch");
  BW_HIP(hipMemcpy(w_host, u->d_w, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
  return BW_OK;
  BWU_GUARD_END
}

extern "C" int bw_unet_set_weights(bw_unet* u, const float* w_host, int64_t n) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(u && w_host, BW_EINVAL, "null argument");
  BW_REQUIRE(n == u->nparam, BW_EINVAL, "parameter count mismatch");
  for (int64_t e = 0; e < n; ++e) BW_REQUIRE(std::isfinite(w_host[e]), BW_EINVAL, "non-finite weight");
  u->w_host.assign(w_host, w_host + n);
  mask_padding(u);
  const size_t nb4 = (size_t)u->nparam * sizeof(float);
  BW_HIP(hipMemset(u->d_m, 0, nb4));
  BW_HIP(hipMemset(u->d_v, 0, nb4));
  u->adam_t = 0;
  upload_weights(u, nullptr);
  return BW_OK;
  BWU_GUARD_END
}

extern "C" int bw_unet_net_forward(bw_unet* u, const int32_t n[3], const float* x, float* y, int32_t nb,
                                   void* stream) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(u && n && x && y, BW_EINVAL, "null argument");
  BW_REQUIRE(nb >= 1, BW_EINVAL, "nb must be >= 1");
  const int nn[3] = {n[0], n[1], n[2]};
  check_grid(nn);
  hipStream_t s = (hipStream_t)stream;
  const Dims d1 = dims_of(n[0], n[1], n[2]);
  Acts a = acts_for(u, d1, nb, false);
  a.X0 = const_cast<float*>(x);
  unet_forward(u, a, d1, nb, s);
  BW_HIP(hipMemcpyAsync(y, a.O, (size_t)nb * d1.V * 16 * sizeof(float), hipMemcpyDeviceToDevice, s));
  BW_HIP(hipGetLastError());
  return BW_OK;
  BWU_GUARD_END
}

extern "C" int bw_unet_net_backward(bw_unet* u, const int32_t n[3], const float* x, const float* dy, float* grad_host,
                                    int32_t nb, void* stream) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(u && n && x && dy && grad_host, BW_EINVAL, "null argument");
  BW_REQUIRE(nb >= 1, BW_EINVAL, "nb must be >= 1");
  const int nn[3] = {n[0], n[1], n[2]};
  check_grid(nn);
  hipStream_t s = (hipStream_t)stream;
  const Dims d1 = dims_of(n[0], n[1], n[2]);
  Acts a = acts_for(u, d1, nb, true);
  a.X0 = const_cast<float*>(x);
  unet_forward(u, a, d1, nb, s);
  BW_HIP(hipMemcpyAsync(a.dO, dy, (size_t)nb * d1.V * 16 * sizeof(float), hipMemcpyDeviceToDevice, s));
  unet_backward(u, a, d1, nb, s);
  hipLaunchKernelGGL(k_mask_grad, dim3(7), dim3(256), 0, s, u->d_g, u->w_off[0], u->w_off[8], u->b_off[8]);
  BW_HIP(hipMemcpyAsync(grad_host, u->d_g, (size_t)u->nparam * sizeof(float), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  return BW_OK;
  BWU_GUARD_END
}

static void check_pair(const bw_unet* u, const bw_rve* r) {
  BW_REQUIRE(r->precision == BW_MIXED, BW_EINVAL, "the learned preconditioner works on BW_MIXED cells");
  BW_REQUIRE(r->device == u->device, BW_EINVAL, "network and cell live on different devices");
  const int nn[3] = {r->g.n0, r->g.n1, r->g.n2};
  check_grid(nn);
}

extern "C" int bw_unet_apply(bw_unet* u, bw_rve* r, const double* k_host, const void* res, void* z, int32_t nrhs,
                             void* stream) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(u && r && k_host && res && z, BW_EINVAL, "null argument");
  BW_REQUIRE(nrhs >= 0, BW_EINVAL, "nrhs < 0");
  BW_REQUIRE(res != z, BW_EINVAL, "r and z must not alias");
  if (nrhs == 0) return BW_OK;
  check_pair(u, r);
  hipStream_t s = (hipStream_t)stream;
  QTable qt = make_qtable(r, k_host, nrhs);
  const double* dq = upload_qtable(r, qt, u->qbuf, s);
  learned_apply(u, r, dq, (const float2*)res, (float2*)z, nrhs, 1.0 / K_scale(r), qt.null_index, s);
  BW_HIP(hipGetLastError());
  BW_HIP(hipStreamSynchronize(s));
  return BW_OK;
  BWU_GUARD_END
}

extern "C" int bw_unet_train_step(bw_unet* u, bw_rve* r, const double* k_host, const void* res, const void* xstar,
                                  int32_t nrhs, double lr, double* loss_host, void* stream) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(u && r && k_host && res && xstar, BW_EINVAL, "null argument");
  BW_REQUIRE(nrhs >= 1, BW_EINVAL, "nrhs must be >= 1");
  BW_REQUIRE(lr >= 0 && std::isfinite(lr), BW_EINVAL, "learning rate must be finite and >= 0");
  check_pair(u, r);
  hipStream_t s = (hipStream_t)stream;
  const Geom& g = r->g;
  const Dims d1 = dims_of(g.n0, g.n1, g.n2);
  const long n3 = 3 * g.nvox;
  QTable qt = make_qtable(r, k_host, nrhs);
  const double* dq = upload_qtable(r, qt, u->qbuf, s);
  Acts a = acts_for(u, d1, nrhs, true);
  Feat f = feat_bufs(u, r, nrhs);
  build_features(r, dq, (const float2*)res, nrhs, 1.0 / K_scale(r), f, a, s);
  // target: normalized real-space image of x* - P^ r (phase and scale of the features)
  float* tgt = (float*)u->tmp.get((size_t)nrhs * g.nvox * (NOUT * sizeof(float) + 3 * sizeof(float2)));
  float2* D = (float2*)(tgt + (size_t)nrhs * g.nvox * NOUT);
  hipLaunchKernelGGL(k_sub, dim3(grid_for(nrhs * n3)), dim3(256), 0, s, (const float2*)xstar, (const float2*)f.Z0, D,
                     (long)nrhs * n3);
  fft3_inplace<true>(r, D, nrhs, s);
  hipLaunchKernelGGL(k_target, dim3(grid_for(nrhs * g.nvox)), dim3(256), 0, s, (const float2*)D, (const double*)f.ps,
                     tgt, g.nvox, nrhs);
  unet_forward(u, a, d1, nrhs, s);
  constexpr int MSE_BLOCKS = 1024;
  double* part = (double*)u->small.get(MSE_BLOCKS * sizeof(double));
  const double scale = 1.0 / ((double)nrhs * g.nvox * NOUT);
  hipLaunchKernelGGL(k_mse, dim3(MSE_BLOCKS), dim3(NT), 0, s, (const float*)a.O, (const float*)tgt, a.dO,
                     (long)nrhs * g.nvox, (float)scale, part);
  unet_backward(u, a, d1, nrhs, s);
  hipLaunchKernelGGL(k_mask_grad, dim3(7), dim3(256), 0, s, u->d_g, u->w_off[0], u->w_off[8], u->b_off[8]);
  u->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)u->adam_t), c2 = 1.f - std::pow(b2, (float)u->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(u->nparam)), dim3(256), 0, s, u->d_w, (const float*)u->d_g, u->d_m, u->d_v,
                     u->nparam, (float)lr, b1, b2, 1e-8f, c1, c2);
  refresh_bf16(u, s);
  std::vector<double> hp(MSE_BLOCKS);
  BW_HIP(hipMemcpyAsync(hp.data(), part, MSE_BLOCKS * sizeof(double), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  double loss = 0;
  for (double v : hp) loss += v;
  if (loss_host) *loss_host = loss * scale;
  BW_REQUIRE(std::isfinite(loss), BW_EINVAL, "training loss is not finite");
  return BW_OK;
  BWU_GUARD_END
}

// One Adam step on the residual loss mean_b ||K z_b - r_b||^2 / ||r_b||^2 with z
// the learned preconditioner applied to r: its gradient with respect to conj z is
// K (K z - r) / ||r||^2 (K is Hermitian), carried back to the network output by
// F^H and the output map (k_outgrad).
extern "C" int bw_unet_train_step_residual(bw_unet* u, bw_rve* r, const double* k_host, const void* res,
                                           int32_t nrhs, double lr, double* loss_host, void* stream) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(u && r && k_host && res, BW_EINVAL, "null argument");
  BW_REQUIRE(nrhs >= 1, BW_EINVAL, "nrhs must be >= 1");
  BW_REQUIRE(lr >= 0 && std::isfinite(lr), BW_EINVAL, "learning rate must be finite and >= 0");
  check_pair(u, r);
  hipStream_t s = (hipStream_t)stream;
  const Geom& g = r->g;
  const Dims d1 = dims_of(g.n0, g.n1, g.n2);
  const long n3 = 3 * g.nvox;
  QTable qt = make_qtable(r, k_host, nrhs);
  const double* dq = upload_qtable(r, qt, u->qbuf, s);
  Acts a = acts_for(u, d1, nrhs, true);
  Feat f = feat_bufs(u, r, nrhs);
  build_features(r, dq, (const float2*)res, nrhs, 1.0 / K_scale(r), f, a, s);
  unet_forward(u, a, d1, nrhs, s);
  float2* Z = (float2*)u->tmp.get((size_t)3 * nrhs * n3 * sizeof(float2));
  float2* E = Z + (size_t)nrhs * n3;
  float2* G = E + (size_t)nrhs * n3;
  float2* W = (float2*)ws<float>(r).work((size_t)nrhs * 6 * g.nvox);
  apply_output(r, f, a, Z, nrhs, s);
  for (int v = 0; v < nrhs; ++v)   // the learned z is zero on the xi + k = 0 voxel
    if (qt.null_index[v] >= 0) zero_voxel<float>((cplx<float>*)Z + (size_t)v * n3, 1, g.nvox, qt.null_index[v], s);
  // E = K z - r (physical units), G = K E / ||r||^2
  launch_apply_K<float>(r, dq, (const cplx<float>*)Z, (cplx<float>*)E, nrhs, K_scale(r), (cplx<float>*)W, s);
  hipLaunchKernelGGL(k_sub, dim3(grid_for(nrhs * n3)), dim3(256), 0, s, (const float2*)E, (const float2*)res, E,
                     (long)nrhs * n3);
  double2* dd = (double2*)u->small.get((size_t)2 * nrhs * sizeof(double2));
  launch_dots<float>((const cplx<float>*)E, (const cplx<float>*)E, nrhs, n3, n3, dd, u->part, nullptr, s);
  launch_dots<float>((const cplx<float>*)res, (const cplx<float>*)res, nrhs, n3, n3, dd + nrhs, r->ws_red2, nullptr, s);
  std::vector<double2> h(2 * nrhs);
  BW_HIP(hipMemcpyAsync(h.data(), dd, (size_t)2 * nrhs * sizeof(double2), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  launch_apply_K<float>(r, dq, (const cplx<float>*)E, (cplx<float>*)G, nrhs, K_scale(r), (cplx<float>*)W, s);
  double loss = 0;
  for (int v = 0; v < nrhs; ++v) {
    BW_REQUIRE(h[nrhs + v].x > 0, BW_EINVAL, "a residual of the batch is zero");
    loss += h[v].x / h[nrhs + v].x;
    scale_vectors<float>((cplx<float>*)G + (size_t)v * n3, (size_t)n3, 1.0 / h[nrhs + v].x, s);
  }
  loss /= nrhs;
  BW_REQUIRE(std::isfinite(loss), BW_EINVAL, "training loss is not finite");
  fft3_inplace<true>(r, G, nrhs, s);           // F^H: the unnormalized inverse transform
  hipLaunchKernelGGL(k_outgrad, dim3(grid_for(nrhs * g.nvox)), dim3(256), 0, s, (const float2*)G,
                     (const double*)f.ps, a.dO, g.nvox, nrhs, (float)(2.0 / nrhs));
  unet_backward(u, a, d1, nrhs, s);
  hipLaunchKernelGGL(k_mask_grad, dim3(7), dim3(256), 0, s, u->d_g, u->w_off[0], u->w_off[8], u->b_off[8]);
  u->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)u->adam_t), c2 = 1.f - std::pow(b2, (float)u->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(u->nparam)), dim3(256), 0, s, u->d_w, (const float*)u->d_g, u->d_m, u->d_v,
                     u->nparam, (float)lr, b1, b2, 1e-8f, c1, c2);
  refresh_bf16(u, s);
  BW_HIP(hipStreamSynchronize(s));
  if (loss_host) *loss_host = loss;
  return BW_OK;
  BWU_GUARD_END
}

namespace bw {

// Flexible preconditioned CG (Polak-Ribiere beta, i.e. one-step K-orthogonal
// directions) on the scaled system K' x = b, with the learned preconditioner
// (u may be null: the plain P^); one wave vector per right-hand side (qt).  Per
// right-hand side, a step whose preconditioned residual is not a descent
// direction (Re <r, z> <= 0 or not finite) takes the plain P^ r instead and
// restarts the direction; after three such steps, or when the residual has not
// dropped by 10% over 10 iterations, that right-hand side continues with the
// plain preconditioner.  x holds the initial guess on entry.
FpcgResult fpcg_run(bw_rve* r, bw_unet* u, const double* dq, const QTable& qt, const float2* bb, float2* xx,
                    int nrhs, double rtol, int maxit, hipStream_t s) {
  const Geom& g = r->g;
  const long n3 = 3 * g.nvox;
  // vectors: r, z, p, Kp, t
  DevBuf& vb = u ? u->vecs : r->ws_misc;
  float2* R = (float2*)vb.get((size_t)5 * nrhs * n3 * sizeof(float2));
  float2* Z = R + (size_t)nrhs * n3;
  float2* P = Z + (size_t)nrhs * n3;
  float2* KP = P + (size_t)nrhs * n3;
  float2* Tt = KP + (size_t)nrhs * n3;
  float2* W = (float2*)ws<float>(r).work((size_t)nrhs * 6 * g.nvox);
  DevBuf& sb = u ? u->small : r->ws_red2;
  DevBuf& scratch = u ? u->part : r->ws_red;
  double2* d_dots = (double2*)sb.get((size_t)nrhs * 4 * sizeof(double2) + (size_t)nrhs * sizeof(int));
  double2* d_coef = d_dots + 2 * nrhs;
  int* d_skip = (int*)(d_coef + 2 * nrhs);
  std::vector<double2> h_dots(2 * nrhs), h_coef(2 * nrhs);
  std::vector<int> h_skip(nrhs, 0);
  auto dots = [&](const float2* X, const float2* Y, double2* out) {
    launch_dots<float>((const cplx<float>*)X, (const cplx<float>*)Y, nrhs, n3, n3, out, scratch, nullptr, s);
  };
  auto fetch = [&](int count) {
    BW_HIP(hipMemcpyAsync(h_dots.data(), d_dots, (size_t)count * nrhs * sizeof(double2), hipMemcpyDeviceToHost, s));
    BW_HIP(hipStreamSynchronize(s));
  };
  auto applyK = [&](const float2* in, float2* out) {
    launch_apply_K<float>(r, dq, (const cplx<float>*)in, (cplx<float>*)out, nrhs, 1.0, (cplx<float>*)W, s);
  };
  const std::vector<int>& nullvec = qt.null_index;
  std::vector<char> plain(nrhs, u ? 0 : 1), active(nrhs, 1);
  std::vector<int> its(nrhs, 0), fb(nrhs, 0);
  std::vector<double> bn(nrhs), rn(nrhs);
  std::vector<std::vector<double>> hist(nrhs);
  auto precondition = [&]() {
    bool any_learned = false;
    for (int v = 0; v < nrhs; ++v) any_learned |= !plain[v] && active[v];
    if (any_learned) {
      learned_apply(u, r, dq, R, Z, nrhs, 1.0, nullvec, s);
      Feat f = feat_bufs(u, r, nrhs);  // f.Z0 holds P^ r of every vector
      for (int v = 0; v < nrhs; ++v)
        if (plain[v])
          BW_HIP(hipMemcpyAsync(Z + (size_t)v * n3, f.Z0 + (size_t)v * n3, n3 * sizeof(float2),
                                hipMemcpyDeviceToDevice, s));
    } else {
      launch_apply_P<float>(r, dq, (const cplx<float>*)R, (cplx<float>*)Z, nrhs, 1.0, s);
    }
  };
  for (int v = 0; v < nrhs; ++v)
    if (qt.null_index[v] >= 0) zero_voxel<float>((cplx<float>*)xx + (size_t)v * n3, 1, g.nvox, qt.null_index[v], s);
  applyK(xx, KP);
  hipLaunchKernelGGL(k_sub, dim3(grid_for(nrhs * n3)), dim3(256), 0, s, bb, (const float2*)KP, R, (long)nrhs * n3);
  dots(bb, bb, d_dots);
  dots(R, R, d_dots + nrhs);
  fetch(2);
  for (int v = 0; v < nrhs; ++v) {
    bn[v] = std::sqrt(h_dots[v].x);
    rn[v] = std::sqrt(h_dots[nrhs + v].x);
    if (rn[v] <= rtol * bn[v]) active[v] = 0;
  }
  int true_checks = 0;
  auto any_active = [&]() {
    for (int v = 0; v < nrhs; ++v)
      if (active[v]) return true;
    return false;
  };
  std::vector<char> restart_v(nrhs, 1);
  while (any_active()) {
    // z = prec(r); descent check; direction update
    precondition();
    dots(R, Z, d_dots);
    dots(KP, Z, d_dots + nrhs);  // KP holds K p of the previous step (unused on restart)
    fetch(2);
    bool need_plain = false;
    std::vector<char> fallback_now(nrhs, 0);
    for (int v = 0; v < nrhs; ++v) {
      if (!active[v] || plain[v]) continue;
      const double rz = h_dots[v].x;
      if (!(rz > 0) || !std::isfinite(rz) || !std::isfinite(h_dots[v].y)) {
        fallback_now[v] = 1;
        need_plain = true;
        if (++fb[v] >= 3) plain[v] = 1;
      }
      auto& h = hist[v];
      if (!plain[v] && h.size() >= 10 && rn[v] > 0.9 * h[h.size() - 10]) {
        plain[v] = 1;
        ++fb[v];
        fallback_now[v] = 1;
        need_plain = true;
      }
    }
    if (need_plain) {
      Feat f = feat_bufs(u, r, nrhs);
      for (int v = 0; v < nrhs; ++v)
        if (fallback_now[v]) {
          BW_HIP(hipMemcpyAsync(Z + (size_t)v * n3, f.Z0 + (size_t)v * n3, n3 * sizeof(float2),
                                hipMemcpyDeviceToDevice, s));
          restart_v[v] = 1;
        }
      dots(KP, Z, d_dots + nrhs);
      fetch(2);
    }
    for (int v = 0; v < nrhs; ++v) {
      h_skip[v] = active[v] ? 0 : 1;
      double2 beta = make_double2(0, 0);
      const double pkp = h_coef[nrhs + v].x;  // <p, Kp> of the previous step
      if (active[v] && !restart_v[v] && pkp > 0) {
        // beta = -<Kp, z> / <p, Kp>
        beta = make_double2(-h_dots[nrhs + v].x / pkp, -h_dots[nrhs + v].y / pkp);
      }
      h_coef[v] = beta;
      restart_v[v] = 0;
    }
    h2d(d_coef, h_coef.data(), (size_t)nrhs * sizeof(double2), s);
    h2d(d_skip, h_skip.data(), (size_t)nrhs * sizeof(int), s);
    hipLaunchKernelGGL(k_fcg_dir, vec_grid(n3, nrhs), dim3(256), 0, s, P, (const float2*)Z, (const double2*)d_coef,
                       (const int*)d_skip, n3);
    // step: alpha = <p, r> / <p, K p>
    applyK(P, KP);
    dots(P, KP, d_dots);
    dots(P, R, d_dots + nrhs);
    fetch(2);
    for (int v = 0; v < nrhs; ++v) {
      double2 alpha = make_double2(0, 0);
      const double pkp = h_dots[v].x;
      if (active[v] && pkp > 0 && std::isfinite(pkp))
        alpha = make_double2(h_dots[nrhs + v].x / pkp, h_dots[nrhs + v].y / pkp);
      h_coef[v] = alpha;
      h_coef[nrhs + v] = make_double2(active[v] ? pkp : 0.0, 0.0);
      if (active[v] && !(pkp > 0)) restart_v[v] = 1;
    }
    h2d(d_coef, h_coef.data(), (size_t)nrhs * sizeof(double2), s);
    hipLaunchKernelGGL(k_fcg_update, vec_grid(n3, nrhs), dim3(256), 0, s, xx, R, (const float2*)P,
                       (const float2*)KP, (const double2*)d_coef, n3);
    dots(R, R, d_dots);
    fetch(1);
    bool check_true = false;
    for (int v = 0; v < nrhs; ++v) {
      if (!active[v]) continue;
      ++its[v];
      hist[v].push_back(rn[v]);
      rn[v] = std::sqrt(h_dots[v].x);
      if (rn[v] <= rtol * bn[v]) check_true = true;
    }
    if (check_true) {
      // replace the recurrence residual by the true one before stopping
      applyK(xx, Tt);
      hipLaunchKernelGGL(k_sub, dim3(grid_for(nrhs * n3)), dim3(256), 0, s, bb, (const float2*)Tt, Tt,
                         (long)nrhs * n3);
      dots(Tt, Tt, d_dots);
      fetch(1);
      ++true_checks;
      for (int v = 0; v < nrhs; ++v) {
        if (!active[v]) continue;
        if (rn[v] > rtol * bn[v]) continue;
        const double tr = std::sqrt(h_dots[v].x);
        if (tr <= rtol * bn[v] || true_checks > 8) {
          active[v] = 0;
        } else {
          BW_HIP(hipMemcpyAsync(R + (size_t)v * n3, Tt + (size_t)v * n3, n3 * sizeof(float2),
                                hipMemcpyDeviceToDevice, s));
          rn[v] = tr;
          restart_v[v] = 1;
        }
      }
    }
    for (int v = 0; v < nrhs; ++v)
      if (active[v] && its[v] >= maxit) active[v] = 0;
  }
  // final true residuals
  applyK(xx, Tt);
  hipLaunchKernelGGL(k_sub, dim3(grid_for(nrhs * n3)), dim3(256), 0, s, bb, (const float2*)Tt, Tt, (long)nrhs * n3);
  dots(Tt, Tt, d_dots);
  fetch(1);
  FpcgResult res;
  res.its = its;
  res.fb = fb;
  res.rel.assign(nrhs, 0.0);
  for (int v = 0; v < nrhs; ++v) {
    res.rel[v] = bn[v] > 0 ? std::sqrt(h_dots[v].x) / bn[v] : 0.0;
    if (!(res.rel[v] <= rtol)) res.conv = false;
    res.total += its[v];
  }
  return res;
}

}  // namespace bw

extern "C" int bw_pcg_solve_learned(bw_rve* r, bw_unet* u, const double k_host[3], const void* b, void* x,
                                    int32_t nrhs, double rtol, int32_t maxit, int32_t* iters_host,
                                    double* relres_host, int32_t* fallbacks_host, void* stream) {
  BWU_GUARD_BEGIN
  BW_REQUIRE(r && k_host && b && x, BW_EINVAL, "null argument");
  BW_REQUIRE(nrhs >= 0, BW_EINVAL, "nrhs < 0");
  BW_REQUIRE(b != x, BW_EINVAL, "b and x must not alias");
  BW_REQUIRE(rtol > 0 && std::isfinite(rtol), BW_EINVAL, "rtol must be > 0");
  if (nrhs == 0) return BW_OK;
  if (u)
    check_pair(u, r);
  else
    BW_REQUIRE(r->precision == BW_MIXED, BW_EINVAL, "flexible PCG works on BW_MIXED cells");
  if (maxit <= 0) maxit = 20000;
  hipStream_t s = (hipStream_t)stream;
  const Geom& g = r->g;
  const long n3 = 3 * g.nvox;
  std::vector<double> ks((size_t)nrhs * 3);
  for (int v = 0; v < nrhs; ++v)
    for (int c = 0; c < 3; ++c) ks[3 * v + c] = k_host[c];
  QTable qt = make_qtable(r, ks.data(), nrhs);
  const int nullv = qt.null_index[0];
  DevBuf& qb = u ? u->qbuf : r->ws_q3;
  const double* dq = upload_qtable(r, qt, qb, s);
  const float2* bb = (const float2*)b;
  float2* xx = (float2*)x;
  if (nullv >= 0) {
    std::vector<float2> vals((size_t)nrhs * 3);
    for (int v = 0; v < nrhs; ++v)
      for (int c = 0; c < 3; ++c)
        BW_HIP(hipMemcpyAsync(&vals[v * 3 + c], bb + ((size_t)v * 3 + c) * g.nvox + nullv, sizeof(float2),
                              hipMemcpyDeviceToHost, s));
    BW_HIP(hipStreamSynchronize(s));
    for (const float2& e : vals)
      BW_REQUIRE(e.x == 0.f && e.y == 0.f, BW_EINVAL, "b has a component on the xi + k = 0 voxel (K is singular)");
  }
  // x' = K_scale x (nondimensional system K' x' = b)
  scale_vectors<float>((cplx<float>*)xx, (size_t)nrhs * n3, K_scale(r), s);
  const FpcgResult res = fpcg_run(r, u, dq, qt, bb, xx, nrhs, rtol, maxit, s);
  scale_vectors<float>((cplx<float>*)xx, (size_t)nrhs * n3, 1.0 / K_scale(r), s);
  BW_HIP(hipStreamSynchronize(s));
  int stalled = 0;
  for (int v = 0; v < nrhs; ++v) {
    if (iters_host) iters_host[v] = res.its[v];
    if (relres_host) relres_host[v] = res.rel[v];
    if (fallbacks_host) fallbacks_host[v] = res.fb[v];
    stalled += res.fb[v] > 0;
  }
  if (!res.conv) {
    set_error("flexible PCG: some right-hand side did not reach rtol");
    return BW_ENOTCONV;
  }
  if (stalled) {
    set_error("flexible PCG: the learned preconditioner stalled for " + std::to_string(stalled) +
              " right-hand side(s), which finished with the plain preconditioner");
    return BW_ESTALL;
  }
  return BW_OK;
  BWU_GUARD_END
}
