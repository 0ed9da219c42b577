// Block kernels of the eigen-solvers (declarations in bw_block.h).
#include "bw_block.h"
#include "bw_ops_impl.h"

namespace bw {

typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
template <typename T> __device__ __forceinline__ cplx<T> from_d2(double2 v);
template <> __device__ __forceinline__ cplx<float> from_d2<float>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ __forceinline__ cplx<double> from_d2<double>(double2 v) { return v; }

// ---------------------------------------------------------------------------
// Gram product on FP64 MFMA (v_mfma_f64_16x16x4f64).
// Lane layout of the instruction (checked on gfx950): A[i][k] from lane
// i + 16 k, B[k][j] from lane j + 16 k, result D[4 r + l / 16][l % 16] in
// register r of lane l.  Re(X^H Y) = Xr^T Yr + Xi^T Yi and
// Im(X^H Y) = Xr^T Yi - Xi^T Yr: four MFMAs per 4-row step and 16x16 block.
// ---------------------------------------------------------------------------
constexpr int GKC = 64;  // rows per wave step (16 MFMA k-steps of 4 rows)

template <typename T>
__global__ __launch_bounds__(256) void k_gram(const cplx<T>* __restrict__ X, int qx, const cplx<T>* __restrict__ Y,
                                              int qy, long n, long vstride, long rows_per_blk,
                                              double* __restrict__ partial) {
  __shared__ double red[4 * 2 * GRAM_QMAX * GRAM_QMAX];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long r0 = (long)blockIdx.x * rows_per_blk;
  const long r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
  const int col = lane & 15, kk = lane >> 4;
  const bool hx0 = col < qx, hx1 = col + 16 < qx, hy0 = col < qy, hy1 = col + 16 < qy;
  const cplx<T>* x0 = X + (size_t)col * vstride;
  const cplx<T>* x1 = X + (size_t)(col + 16) * vstride;
  const cplx<T>* y0 = Y + (size_t)col * vstride;
  const cplx<T>* y1 = Y + (size_t)(col + 16) * vstride;
  d4_t accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = d4_t{0, 0, 0, 0};
      acci[a][b] = d4_t{0, 0, 0, 0};
    }
  // the four waves interleave 4-row steps; operands come straight from global
  // memory (consecutive steps of a wave reuse the same cache lines)
  for (long e0 = r0 + wave * 4; e0 < r1; e0 += 16 * 4) {
    double2 a[4][2], bb[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long e = e0 + (long)u * 16 + kk;
      const bool in = e < r1;
      a[u][0] = (in && hx0) ? to_d2(x0[e]) : make_double2(0, 0);
      a[u][1] = (in && hx1) ? to_d2(x1[e]) : make_double2(0, 0);
      bb[u][0] = (in && hy0) ? to_d2(y0[e]) : make_double2(0, 0);
      bb[u][1] = (in && hy1) ? to_d2(y1[e]) : make_double2(0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int bp = 0; bp < 2; ++bp)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          if ((bp == 1 && qx <= 16) || (bj == 1 && qy <= 16)) continue;
          const double2 av = a[u][bp], bv = bb[u][bj];
          accr[bp][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, accr[bp][bj], 0, 0, 0);
          accr[bp][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.y, accr[bp][bj], 0, 0, 0);
          acci[bp][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, acci[bp][bj], 0, 0, 0);
          acci[bp][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.x, acci[bp][bj], 0, 0, 0);
        }
  }
  // sum the four waves' partial blocks through LDS
  const int nq = qx * qy;
#pragma unroll
  for (int bp = 0; bp < 2; ++bp)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = bp * 16 + 4 * r + (lane >> 4), j = bj * 16 + (lane & 15);
        if (i < qx && j < qy) {
          red[((size_t)wave * nq + i * qy + j) * 2] = accr[bp][bj][r];
          red[((size_t)wave * nq + i * qy + j) * 2 + 1] = acci[bp][bj][r];
        }
      }
  __syncthreads();
  for (int t = tid; t < 2 * nq; t += 256)
    partial[(size_t)blockIdx.x * 2 * nq + t] = red[t] + red[2 * nq + t] + red[4 * nq + t] + red[6 * nq + t];
}

// second phase of the Gram product: one workgroup per matrix entry sums the
// per-block partials in block order
__global__ __launch_bounds__(256) void k_gram_finalize(const double* __restrict__ partial, int nblk, int n2q,
                                                       double* __restrict__ G) {
  __shared__ double sh[4];
  const int t = blockIdx.x;
  double acc = 0;
  for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[(size_t)b * n2q + t];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) G[t] = acc;
}

template <typename T>
void launch_gram(const cplx<T>* X, int qx, const cplx<T>* Y, int qy, long n, long vstride, double2* G,
                 DevBuf& scratch, unsigned* counter, hipStream_t s) {
  BW_REQUIRE(qx >= 1 && qy >= 1 && qx <= GRAM_QMAX && qy <= GRAM_QMAX, BW_EINVAL, "Gram block exceeds 32 vectors");
  long nblk = (n + 4 * GKC - 1) / (4 * GKC);
  if (nblk > 512) nblk = 512;
  if (nblk < 1) nblk = 1;
  long rows = (n + nblk - 1) / nblk;
  rows = (rows + GKC - 1) / GKC * GKC;
  nblk = (n + rows - 1) / rows;
  const size_t part_bytes = (size_t)nblk * 2 * qx * qy * sizeof(double);
  char* base = (char*)scratch.get(part_bytes);
  BW_LAUNCH("k_gram_mfma", (long)qx * qy, (k_gram<T>), dim3((unsigned)nblk), dim3(256), 0, s, X, qx, Y, qy, n,
            vstride, rows, (double*)base);
  const int n2q = 2 * qx * qy;
  hipLaunchKernelGGL(k_gram_finalize, dim3(n2q), dim3(256), 0, s, (const double*)base, (int)nblk, n2q, (double*)G);
  (void)counter;
}

// ---------------------------------------------------------------------------
// Ritz update Y_j = sum_p X_p Q[p][j]
// ---------------------------------------------------------------------------
// Y[:, j] = sum_p X[:, p] Q[p][j] (FP64 accumulation).  The coefficients are
// the same for every lane, so they are read with scalar loads; QO bounds qout
// at compile time (fewer accumulators, higher occupancy).  RQ: real
// coefficients (the eigenvectors of the real symmetric Lanczos matrices), two
// multiply-adds per term instead of four: the update is then bound by memory,
// not by FP64 issue.
template <typename T, int QO, bool RQ = false>
__global__ __launch_bounds__(256) void k_ritz(const cplx<T>* __restrict__ X, int q, const double2* __restrict__ Q,
                                              int ldq, cplx<T>* __restrict__ Y, int qout, long n, long vstride) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    double2 acc[QO];
#pragma unroll
    for (int j = 0; j < QO; ++j) acc[j] = make_double2(0, 0);
#pragma unroll 2
    for (int p = 0; p < q; ++p) {
      const double2 x = to_d2(X[(size_t)p * vstride + e]);
      const double2* __restrict__ Qp = Q + (size_t)p * ldq;
#pragma unroll
      for (int j = 0; j < QO; ++j) {
        // columns past qout take coefficient 0 (a uniform select, not a branch,
        // so the coefficients stay scalar loads in batches)
        if (RQ) {
          double c = Qp[j < qout ? j : qout - 1].x;
          if (j >= qout) c = 0.0;
          acc[j].x += x.x * c;
          acc[j].y += x.y * c;
        } else {
          double2 c = Qp[j < qout ? j : qout - 1];
          if (j >= qout) c = make_double2(0.0, 0.0);
          acc[j].x += x.x * c.x - x.y * c.y;
          acc[j].y += x.x * c.y + x.y * c.x;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < QO; ++j)
      if (j < qout) Y[(size_t)j * vstride + e] = from_d2<T>(acc[j]);
  }
}

template <typename T>
void launch_ritz(const cplx<T>* X, int q, const double2* Q, int ldq, cplx<T>* Y, int qout, long n, long vstride,
                 hipStream_t s, bool real_q) {
  BW_REQUIRE(q <= GEIG_QMAX && qout <= GRAM_QMAX, BW_EINVAL, "Ritz block too large");
  long nb = (n + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (real_q) {
    // the Lanczos sizes (14 refined, 18 kept for 12 wanted modes) get buckets of
    // their own: no multiply-adds on padding columns
    auto go = [&](auto qo) {
      constexpr int QO = decltype(qo)::value;
      BW_LAUNCH("k_ritz", (long)q * qout, (k_ritz<T, QO, true>), dim3((unsigned)nb), dim3(256), 0, s, X, q, Q, ldq,
                Y, qout, n, vstride);
    };
    if (qout <= 8) go(std::integral_constant<int, 8>{});
    else if (qout <= 14) go(std::integral_constant<int, 14>{});
    else if (qout <= 18) go(std::integral_constant<int, 18>{});
    else if (qout <= 24) go(std::integral_constant<int, 24>{});
    else go(std::integral_constant<int, GRAM_QMAX>{});
    return;
  }
  if (qout <= 8)
    BW_LAUNCH("k_ritz", (long)q * qout, (k_ritz<T, 8>), dim3((unsigned)nb), dim3(256), 0, s, X, q, Q, ldq, Y, qout, n,
              vstride);
  else if (qout <= 16)
    BW_LAUNCH("k_ritz", (long)q * qout, (k_ritz<T, 16>), dim3((unsigned)nb), dim3(256), 0, s, X, q, Q, ldq, Y, qout,
              n, vstride);
  else if (qout <= 24)
    BW_LAUNCH("k_ritz", (long)q * qout, (k_ritz<T, 24>), dim3((unsigned)nb), dim3(256), 0, s, X, q, Q, ldq, Y, qout,
              n, vstride);
  else
    BW_LAUNCH("k_ritz", (long)q * qout, (k_ritz<T, GRAM_QMAX>), dim3((unsigned)nb), dim3(256), 0, s, X, q, Q, ldq, Y,
              qout, n, vstride);
}

// ---------------------------------------------------------------------------
// batched inner products
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_dots(const cplx<T>* __restrict__ X, const cplx<T>* __restrict__ Y, long n,
                                             long vstride, int bpv, double* partial, int maxb) {
  __shared__ double sh[NT / 64];
  const int p = blockIdx.x / bpv;
  const int b = blockIdx.x - p * bpv;
  double sr = 0, si = 0;
  for (long e = (long)b * NT + threadIdx.x; e < n; e += (long)bpv * NT) {
    const double2 x = to_d2(X[(size_t)p * vstride + e]);
    const double2 y = to_d2(Y[(size_t)p * vstride + e]);
    sr += x.x * y.x + x.y * y.y;
    si += x.x * y.y - x.y * y.x;
  }
  const double vals[2] = {sr, si};
  store_partials<2>(vals, partial, p, b, maxb, sh);
}

__global__ __launch_bounds__(NT) void k_dots_finalize(const double* __restrict__ partial, int bpv, double2* out) {
  __shared__ double sh[NT / 64];
  double tot[2];
  sum_partials<2>(tot, partial, blockIdx.x, bpv, bpv, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = make_double2(tot[0], tot[1]);
}

template <typename T>
void launch_dots(const cplx<T>* X, const cplx<T>* Y, int nv, long n, long vstride, double2* out, DevBuf& scratch,
                 unsigned* counters, hipStream_t s) {
  BW_REQUIRE(nv <= 256, BW_EINVAL, "too many vectors for one dot-product launch");
  const int bpv = pw_blocks(n);
  const size_t part_bytes = (size_t)nv * bpv * 2 * sizeof(double);
  char* base = (char*)scratch.get(part_bytes);
  hipLaunchKernelGGL((k_dots<T>), dim3(nv * bpv), dim3(NT), 0, s, X, Y, n, vstride, bpv, (double*)base, bpv);
  hipLaunchKernelGGL(k_dots_finalize, dim3(nv), dim3(NT), 0, s, (const double*)base, bpv, out);
  (void)counters;
}

// ---------------------------------------------------------------------------
// vector utilities
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_lincomb(const cplx<T>* __restrict__ A, const cplx<T>* __restrict__ B, const double* __restrict__ lam,
                          cplx<T>* __restrict__ R, long n, long vstride) {
  const int p = blockIdx.y;
  const double l = lam[p];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double2 a = to_d2(A[(size_t)p * vstride + e]), b = to_d2(B[(size_t)p * vstride + e]);
    R[(size_t)p * vstride + e] = from_d2<T>(make_double2(a.x - l * b.x, a.y - l * b.y));
  }
}

template <typename T>
void launch_lincomb(const cplx<T>* A, const cplx<T>* B, const double* lam, cplx<T>* R, int nv, long n, long vstride,
                    hipStream_t s) {
  if (nv <= 0) return;
  long nb = (n + 255) / 256;
  if (nb > 512) nb = 512;
  hipLaunchKernelGGL((k_lincomb<T>), dim3((unsigned)nb, nv), dim3(256), 0, s, A, B, lam, R, n, vstride);
}

template <typename T>
__global__ void k_scale_cols(const cplx<T>* __restrict__ X, const double* __restrict__ sc, cplx<T>* __restrict__ Y,
                             long n, long vstride) {
  const int p = blockIdx.y;
  const double f = sc[p];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double2 a = to_d2(X[(size_t)p * vstride + e]);
    Y[(size_t)p * vstride + e] = from_d2<T>(make_double2(a.x * f, a.y * f));
  }
}

template <typename T>
void launch_scale_cols(const cplx<T>* X, const double* sc, cplx<T>* Y, int nv, long n, long vstride, hipStream_t s) {
  if (nv <= 0) return;
  long nb = (n + 255) / 256;
  if (nb > 512) nb = 512;
  hipLaunchKernelGGL((k_scale_cols<T>), dim3((unsigned)nb, nv), dim3(256), 0, s, X, sc, Y, n, vstride);
}

template <typename TS, typename TD>
__global__ void k_convert(const cplx<TS>* __restrict__ src, cplx<TD>* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = from_d2<TD>(to_d2(src[i]));
}

template <typename TS, typename TD>
void launch_convert(const cplx<TS>* src, cplx<TD>* dst, size_t n, hipStream_t s) {
  if (n == 0) return;
  size_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL((k_convert<TS, TD>), dim3((unsigned)nb), dim3(256), 0, s, src, dst, n);
}

// Gamma deflation, step 1: a_c = MX_p(c, j*) / MN_c(c, j*), X_p(c, j*) -= a_c
template <typename T>
__global__ void k_deflate_coef(cplx<T>* X, const cplx<T>* MX, const cplx<T>* MN, int nv, long nvox, long jstar,
                               double2* coef) {
  const int t = threadIdx.x;
  if (t >= nv * 3) return;
  const int p = t / 3, c = t - 3 * p;
  const double2 m = to_d2(MX[((size_t)p * 3 + c) * nvox + jstar]);
  const double2 d = to_d2(MN[((size_t)c * 3 + c) * nvox + jstar]);
  const double den = d.x * d.x + d.y * d.y;
  const double2 a = make_double2((m.x * d.x + m.y * d.y) / den, (m.y * d.x - m.x * d.y) / den);
  coef[t] = a;
  const double2 x = to_d2(X[((size_t)p * 3 + c) * nvox + jstar]);
  X[((size_t)p * 3 + c) * nvox + jstar] = from_d2<T>(make_double2(x.x - a.x, x.y - a.y));
}

// step 2: MX_p(c, :) -= a_c MN_c(c, :)
template <typename T>
__global__ void k_deflate_apply(cplx<T>* MX, const cplx<T>* MN, long nvox, const double2* coef) {
  const int p = blockIdx.y / 3, c = blockIdx.y - 3 * (blockIdx.y / 3);
  const double2 a = coef[p * 3 + c];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nvox; e += (long)gridDim.x * blockDim.x) {
    const double2 mn = to_d2(MN[((size_t)c * 3 + c) * nvox + e]);
    const double2 m = to_d2(MX[((size_t)p * 3 + c) * nvox + e]);
    MX[((size_t)p * 3 + c) * nvox + e] =
        from_d2<T>(make_double2(m.x - (a.x * mn.x - a.y * mn.y), m.y - (a.x * mn.y + a.y * mn.x)));
  }
}

template <typename T>
void launch_deflate(cplx<T>* X, cplx<T>* MX, const cplx<T>* MN, int nv, long nvox, long jstar, double2* coef,
                    hipStream_t s) {
  BW_REQUIRE(nv * 3 <= 256, BW_EINVAL, "deflation block too large");
  hipLaunchKernelGGL((k_deflate_coef<T>), dim3(1), dim3(256), 0, s, X, (const cplx<T>*)MX, MN, nv, nvox, jstar, coef);
  long nb = (nvox + 255) / 256;
  if (nb > 256) nb = 256;
  hipLaunchKernelGGL((k_deflate_apply<T>), dim3((unsigned)nb, nv * 3), dim3(256), 0, s, MX, MN, nvox,
                     (const double2*)coef);
}

template <typename T>
__global__ void k_planewaves(cplx<T>* U, int nv, long nvox, const long* vox, const double* pol) {
  const int t = threadIdx.x;
  if (t >= nv * 3) return;
  const int p = t / 3, c = t - 3 * p;
  U[((size_t)p * 3 + c) * nvox + vox[p]] = from_d2<T>(make_double2(pol[t], 0.0));
}

template <typename T>
void launch_planewaves(cplx<T>* U, int nv, long nvox, const long* vox, const double* pol, hipStream_t s) {
  BW_REQUIRE(nv * 3 <= 256, BW_EINVAL, "too many start vectors");
  BW_HIP(hipMemsetAsync(U, 0, (size_t)nv * 3 * nvox * sizeof(cplx<T>), s));
  hipLaunchKernelGGL((k_planewaves<T>), dim3(1), dim3(256), 0, s, U, nv, nvox, vox, pol);
}

// ---------------------------------------------------------------------------
// small generalized Hermitian eigenproblem, one workgroup of 64 threads:
// diagonal scaling, Cholesky of Mq, A = L^-1 Kq L^-H, cyclic Jacobi with the
// round-robin ordering (q/2 disjoint rotations per step), Q = D L^-H Z.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmc(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

__global__ __launch_bounds__(64) void k_small_geig(const double2* __restrict__ Kq_all,
                                                   const double2* __restrict__ Mq_all, int q, double* lam_all,
                                                   double2* Qout_all, int* info_all, int m_identity) {
  // one workgroup per problem of the batch
  const double2* Kq = Kq_all + (size_t)blockIdx.x * q * q;
  const double2* Mq = Mq_all + (size_t)blockIdx.x * q * q;
  double* lam = lam_all + (size_t)blockIdx.x * q;
  double2* Qout = Qout_all + (size_t)blockIdx.x * q * q;
  int* info = info_all + blockIdx.x;
  constexpr int QE = GEIG_QMAX;
  __shared__ double2 A[QE * QE];
  __shared__ double2 Z[QE * QE];
  __shared__ double2 Lm[QE * QE];
  __shared__ double dsc[QE];
  __shared__ double rc[QE / 2], rs[QE / 2];
  __shared__ double2 rph[QE / 2];
  __shared__ int rp[QE / 2], rq[QE / 2], perm[QE];
  __shared__ int flag;
  const int tid = threadIdx.x;
  if (tid == 0) {
    flag = 0;
    info[0] = 0;
  }
  for (int i = tid; i < q; i += 64) dsc[i] = m_identity ? 1.0 : 1.0 / sqrt(Mq[i * q + i].x);
  __syncthreads();
  for (int idx = tid; idx < q * q; idx += 64) {
    const int i = idx / q, j = idx - i * q;
    const double s = dsc[i] * dsc[j];
    const double2 k1 = Kq[i * q + j], k2 = Kq[j * q + i];
    A[idx] = make_double2(0.5 * (k1.x + k2.x) * s, 0.5 * (k1.y - k2.y) * s);  // Hermitian part
    if (m_identity) {
      Lm[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    } else {
      const double2 m1 = Mq[i * q + j], m2 = Mq[j * q + i];
      Lm[idx] = make_double2(0.5 * (m1.x + m2.x) * s, 0.5 * (m1.y - m2.y) * s);
    }
  }
  __syncthreads();
  // Cholesky Lm = L L^H (lower), in place
  for (int j = 0; j < q; ++j) {
    if (tid == 0) {
      double d = Lm[j * q + j].x;
      for (int k = 0; k < j; ++k) d -= Lm[j * q + k].x * Lm[j * q + k].x + Lm[j * q + k].y * Lm[j * q + k].y;
      if (!(d > 0)) {
        flag = 1;
        d = 1e-300;
      }
      Lm[j * q + j] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < q; i += 64) {
      double2 v = Lm[i * q + j];
      for (int k = 0; k < j; ++k) {
        const double2 t = cmc(Lm[i * q + k], Lm[j * q + k]);
        v.x -= t.x;
        v.y -= t.y;
      }
      const double inv = 1.0 / Lm[j * q + j].x;
      Lm[i * q + j] = make_double2(v.x * inv, v.y * inv);
    }
    __syncthreads();
  }
  if (tid == 0 && flag) info[0] = 1;
  // B = L^-1 A (column c per thread), kept in Z
  for (int c = tid; c < q; c += 64) {
    for (int i = 0; i < q; ++i) {
      double2 v = A[i * q + c];
      for (int k = 0; k < i; ++k) {
        const double2 t = cm(Lm[i * q + k], Z[k * q + c]);
        v.x -= t.x;
        v.y -= t.y;
      }
      const double inv = 1.0 / Lm[i * q + i].x;
      Z[i * q + c] = make_double2(v.x * inv, v.y * inv);
    }
  }
  __syncthreads();
  // A = B L^-H: column c of C = L^-1 B^H gives row c of A = C^H
  for (int c = tid; c < q; c += 64) {
    for (int i = 0; i < q; ++i) {
      const double2 b = Z[c * q + i];
      double2 v = make_double2(b.x, -b.y);
      for (int k = 0; k < i; ++k) {
        const double2 ck = A[c * q + k];  // A[c][k] holds conj(C[k][c])
        const double2 t = cm(Lm[i * q + k], make_double2(ck.x, -ck.y));
        v.x -= t.x;
        v.y -= t.y;
      }
      const double inv = 1.0 / Lm[i * q + i].x;
      A[c * q + i] = make_double2(v.x * inv, -v.y * inv);
    }
  }
  __syncthreads();
  for (int idx = tid; idx < q * q; idx += 64) {
    const int i = idx / q, j = idx - i * q;
    Z[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int idx = tid; idx < q * q; idx += 64) {  // re-Hermitize
    const int i = idx / q, j = idx - i * q;
    if (i < j) {
      const double2 a = A[i * q + j], b = A[j * q + i];
      const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      A[i * q + j] = h;
      A[j * q + i] = make_double2(h.x, -h.y);
    } else if (i == j) {
      A[idx].y = 0.0;
    }
  }
  __syncthreads();
  const int m = (q + 1) & ~1;
  const int npair = m / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) {
      double off = 0, dia = 0;
      for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
          const double v = A[i * q + j].x * A[i * q + j].x + A[i * q + j].y * A[i * q + j].y;
          if (i == j)
            dia += v;
          else
            off += v;
        }
      flag = off <= 1e-30 * dia ? 1 : 0;
    }
    __syncthreads();
    if (flag) break;
    for (int step = 0; step < m - 1; ++step) {
      if (tid < npair) {
        int a, b;
        if (tid == 0) {
          a = m - 1;
          b = step;
        } else {
          a = (step + tid) % (m - 1);
          b = (step - tid + (m - 1)) % (m - 1);
        }
        int p = a < b ? a : b, qq = a < b ? b : a;
        double cs = 1.0, sn = 0.0;
        double2 ph = make_double2(1.0, 0.0);
        if (qq < q) {
          const double2 c = A[p * q + qq];
          const double ac = sqrt(c.x * c.x + c.y * c.y);
          const double app = A[p * q + p].x, aqq = A[qq * q + qq].x;
          if (ac > 1e-300 && ac > 1e-18 * (fabs(app) + fabs(aqq))) {
            ph = make_double2(c.x / ac, c.y / ac);
            const double tau = (aqq - app) / (2.0 * ac);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            cs = 1.0 / sqrt(1.0 + t * t);
            sn = t * cs;
          }
        } else {
          qq = p;  // dummy partner: identity
        }
        rp[tid] = p;
        rq[tid] = qq;
        rc[tid] = cs;
        rs[tid] = sn;
        rph[tid] = ph;
      }
      __syncthreads();
      // rows: A <- J^H A
      for (int w = tid; w < npair * q; w += 64) {
        const int i = w / q, j = w - i * q;
        const int p = rp[i], qq = rq[i];
        if (p == qq || rs[i] == 0.0) continue;
        const double cs = rc[i], sn = rs[i];
        const double2 ph = rph[i];
        const double2 ap = A[p * q + j], aq = A[qq * q + j];
        const double2 e = cm(ph, aq);  // e^{i phi} a_q
        A[p * q + j] = make_double2(cs * ap.x - sn * e.x, cs * ap.y - sn * e.y);
        A[qq * q + j] = make_double2(sn * ap.x + cs * e.x, sn * ap.y + cs * e.y);
      }
      __syncthreads();
      // columns: A <- A J, Z <- Z J
      for (int w = tid; w < npair * q; w += 64) {
        const int i = w / q, j = w - i * q;
        const int p = rp[i], qq = rq[i];
        if (p == qq || rs[i] == 0.0) continue;
        const double cs = rc[i], sn = rs[i];
        const double2 phc = make_double2(rph[i].x, -rph[i].y);
        {
          const double2 ap = A[j * q + p], aq = A[j * q + qq];
          const double2 e = cm(phc, aq);
          A[j * q + p] = make_double2(cs * ap.x - sn * e.x, cs * ap.y - sn * e.y);
          A[j * q + qq] = make_double2(sn * ap.x + cs * e.x, sn * ap.y + cs * e.y);
        }
        {
          const double2 zp = Z[j * q + p], zq = Z[j * q + qq];
          const double2 e = cm(phc, zq);
          Z[j * q + p] = make_double2(cs * zp.x - sn * e.x, cs * zp.y - sn * e.y);
          Z[j * q + qq] = make_double2(sn * zp.x + cs * e.x, sn * zp.y + cs * e.y);
        }
      }
      __syncthreads();
    }
  }
  // sort eigenvalues ascending
  if (tid == 0) {
    for (int i = 0; i < q; ++i) perm[i] = i;
    for (int i = 0; i < q; ++i) {
      int best = i;
      for (int j = i + 1; j < q; ++j)
        if (A[perm[j] * q + perm[j]].x < A[perm[best] * q + perm[best]].x) best = j;
      const int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
  }
  __syncthreads();
  // Q = D L^-H Z (back substitution per column)
  for (int c = tid; c < q; c += 64) {
    const int src = perm[c];
    lam[c] = A[src * q + src].x;
    for (int i = q - 1; i >= 0; --i) {
      double2 v = Z[i * q + src];
      for (int k = i + 1; k < q; ++k) {
        // conj(L[k][i]) * X[k]
        const double2 l = Lm[k * q + i];
        const double2 x = A[k * q + src];  // A column src reused as scratch for X
        v.x -= l.x * x.x + l.y * x.y;
        v.y -= l.x * x.y - l.y * x.x;
      }
      const double inv = 1.0 / Lm[i * q + i].x;
      A[i * q + src] = make_double2(v.x * inv, v.y * inv);
    }
    for (int i = 0; i < q; ++i) {
      const double2 x = A[i * q + src];
      Qout[i * q + c] = make_double2(x.x * dsc[i], x.y * dsc[i]);
    }
  }
}

void launch_small_geig(const double2* Kq, const double2* Mq, int q, double* lam, double2* Q, int* info,
                       hipStream_t s) {
  BW_REQUIRE(q >= 1 && q <= GEIG_QMAX, BW_EINVAL, "small eigenproblem larger than 48");
  hipLaunchKernelGGL(k_small_geig, dim3(1), dim3(64), 0, s, Kq, Mq, q, lam, Q, info, 0);
}

void launch_small_eig_batched(const double2* H, int q, int nb, double* lam, double2* Q, int* info, hipStream_t s) {
  BW_REQUIRE(q >= 1 && q <= GEIG_QMAX, BW_EINVAL, "small eigenproblem larger than 48");
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_small_geig, dim3(nb), dim3(64), 0, s, H, H, q, lam, Q, info, 1);
}

// ---------------------------------------------------------------------------
// batched per-k basis products (Lanczos)
// ---------------------------------------------------------------------------
// Work units for the kernel timing: J basis vectors per active wave vector (the
// activity flags are read back only while timing is on).
static long active_units(const int* act, int nk, int J, hipStream_t s) {
  if (!timing_enabled()) return 0;
  std::vector<int> a(nk, 1);
  if (act) {
    BW_HIP(hipMemcpyAsync(a.data(), act, nk * sizeof(int), hipMemcpyDeviceToHost, s));
    BW_HIP(hipStreamSynchronize(s));
  }
  long u = 0;
  for (int k = 0; k < nk; ++k) u += a[k] ? J : 0;
  return u;
}

// Products of each basis vector with two right-hand vectors at once (the
// delayed re-orthogonalization of the Lanczos process): out0[k, i] = <X_k[i],
// Y0_k>, out1[k, i] = <X_k[i], Y1_k>, reading every basis vector once.
// I: the index type of the element offsets (32-bit when 8 xi + n < 2^32).
template <typename T, typename I>
__global__ __launch_bounds__(NT) void k_mdot8x2(const cplx<T>* __restrict__ X, long xk, long xi, int J,
                                                const cplx<T>* __restrict__ Y0, long yk0,
                                                const cplx<T>* __restrict__ Y1, long yk1, long n, const int* act,
                                                double* partial, int bpv) {
  __shared__ double sh[32][NT / 64];
  const int b = blockIdx.x, g = blockIdx.y, k = blockIdx.z;
  if (act && !act[k]) return;
  const int i0 = 8 * g;
  const int ni = J - i0 < 8 ? J - i0 : 8;
  const cplx<T>* x = X + (size_t)k * xk + (size_t)i0 * xi;
  const cplx<T>* y0 = Y0 + (size_t)k * yk0;
  const cplx<T>* y1 = Y1 + (size_t)k * yk1;
  double a0r[8], a0i[8], a1r[8], a1i[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a0r[i] = a0i[i] = a1r[i] = a1i[i] = 0.0;
  // two elements of the thread's sequence per pass, all their loads issued
  // first; the terms are added in the same element order as one at a time
  const I st = (I)bpv * NT, xs = (I)xi;
  for (I e = (I)b * NT + threadIdx.x; e < (I)n; e += 2 * st) {
    const bool two = e + st < (I)n;
    cplx<T> r0[2], r1[2], av[2][8];     // held as loaded, widened at use
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      const I eu = e + u * st;
      r0[u] = y0[eu];
      r1[u] = y1[eu];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < ni) av[u][i] = x[(I)i * xs + eu];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      const double2 c0 = to_d2(r0[u]), c1 = to_d2(r1[u]);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (i < ni) {
          const double2 a = to_d2(av[u][i]);
          a0r[i] += a.x * c0.x + a.y * c0.y;
          a0i[i] += a.x * c0.y - a.y * c0.x;
          a1r[i] += a.x * c1.x + a.y * c1.y;
          a1i[i] += a.x * c1.y - a.y * c1.x;
        }
      }
    }
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double r0 = wave_sum(a0r[i]), r1 = wave_sum(a0i[i]), r2 = wave_sum(a1r[i]), r3 = wave_sum(a1i[i]);
    if (l == 0) {
      sh[4 * i][w] = r0;
      sh[4 * i + 1][w] = r1;
      sh[4 * i + 2][w] = r2;
      sh[4 * i + 3][w] = r3;
    }
  }
  __syncthreads();
  const int v = threadIdx.x;
  if (v < 4 * ni) {
    double acc = 0;
    for (int ww = 0; ww < NT / 64; ++ww) acc += sh[v][ww];
    partial[((size_t)(k * J + i0 + (v >> 2)) * bpv + b) * 4 + (v & 3)] = acc;
  }
}

__global__ __launch_bounds__(NT) void k_mdot2_finalize(const double* __restrict__ partial, int bpv, int J,
                                                       const int* act, double2* out0, double2* out1, int ldo) {
  __shared__ double sh[NT / 64];
  const int idx = blockIdx.x;  // k * J + i
  const int k = idx / J, i = idx - k * J;
  if (act && !act[k]) return;
  double tot[4];
  sum_partials<4>(tot, partial, idx, bpv, bpv, sh);
  if (threadIdx.x == 0) {
    out0[(size_t)k * ldo + i] = make_double2(tot[0], tot[1]);
    out1[(size_t)k * ldo + i] = make_double2(tot[2], tot[3]);
  }
}

template <typename T>
void launch_mdot2(const cplx<T>* X, long xk, long xi, int J, const cplx<T>* Y0, long yk0, const cplx<T>* Y1, long yk1,
                  int nk, long n, const int* act, double2* out0, double2* out1, int ldo, DevBuf& scratch,
                  hipStream_t s) {
  if (J <= 0 || nk <= 0) return;
  int bpv = pw_blocks(n);
  if (bpv > 256) bpv = 256;
  double* partial = (double*)scratch.get((size_t)nk * J * bpv * 4 * sizeof(double));
  if (8.0 * xi + n < 4294967296.0)
    BW_LAUNCH("k_mdot2", active_units(act, nk, J, s), (k_mdot8x2<T, uint32_t>), dim3(bpv, (J + 7) / 8, nk), dim3(NT),
              0, s, X, xk, xi, J, Y0, yk0, Y1, yk1, n, act, partial, bpv);
  else
    BW_LAUNCH("k_mdot2", active_units(act, nk, J, s), (k_mdot8x2<T, size_t>), dim3(bpv, (J + 7) / 8, nk), dim3(NT),
              0, s, X, xk, xi, J, Y0, yk0, Y1, yk1, n, act, partial, bpv);
  hipLaunchKernelGGL(k_mdot2_finalize, dim3(nk * J), dim3(NT), 0, s, (const double*)partial, bpv, J, act, out0, out1,
                     ldo);
}

// The delayed re-orthogonalization update of one Lanczos step, one pass over
// the J finished basis vectors X_k[0..J-1]:
//   Y0_k <- f0 Y0_k - sum_i X_k[i] a_i                 (the pending vector, finished)
//   Y1_k <- f1 Y1_k - sum_i X_k[i] b_i - g Y0_k(new)    (the new direction, once orthogonalized)
// Coefficients of wave vector k at c + k * ldc: a[0..J-1], b[0..J-1], then
// (f0, 0), (f1, 0), g.  Y1 == nullptr: the first output only.  FP64 accumulation.
// I: the index type of the element offsets (32-bit when J xi + n < 2^32: a
// uniform base plus a 32-bit lane offset per load, no 64-bit address).
template <typename T, typename I>
__global__ __launch_bounds__(256) void k_mlincomb2(cplx<T>* __restrict__ Y0, long yk0, cplx<T>* __restrict__ Y1,
                                                   long yk1, const cplx<T>* __restrict__ X, long xk, long xi, int J,
                                                   const double2* __restrict__ c, int ldc, long n, const int* act) {
  const int k = blockIdx.z;
  if (act && !act[k]) return;
  const cplx<T>* x = X + (size_t)k * xk;
  cplx<T>* y0 = Y0 + (size_t)k * yk0;
  cplx<T>* y1 = Y1 ? Y1 + (size_t)k * yk1 : nullptr;
  const double2* ck = c + (size_t)k * ldc;
  const double f0 = ck[2 * J].x, f1 = ck[2 * J + 1].x;
  const double2 gg = ck[2 * J + 2];
  const I xs = (I)xi;
  for (I e = (I)blockIdx.x * 256 + threadIdx.x; e < (I)n; e += (I)gridDim.x * 256) {
    double ar = 0, ai = 0, br = 0, bi = 0;
    auto term = [&](const double2 v, int i) {
      const double2 ca = ck[i];
      ar += v.x * ca.x - v.y * ca.y;
      ai += v.x * ca.y + v.y * ca.x;
      if (y1) {
        const double2 cb = ck[J + i];
        br += v.x * cb.x - v.y * cb.y;
        bi += v.x * cb.y + v.y * cb.x;
      }
    };
    // sixteen basis loads in flight at a time (held as loaded, widened at use);
    // the terms are still added in the order i = 0, 1, ..., so the sums do not
    // change
    int i = 0;
    for (; i + 16 <= J; i += 16) {
      cplx<T> v[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) v[t] = x[(I)(i + t) * xs + e];
#pragma unroll
      for (int t = 0; t < 16; ++t) term(to_d2(v[t]), i + t);
    }
    for (; i + 4 <= J; i += 4) {
      cplx<T> v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t] = x[(I)(i + t) * xs + e];
#pragma unroll
      for (int t = 0; t < 4; ++t) term(to_d2(v[t]), i + t);
    }
    for (; i < J; ++i) term(to_d2(x[(I)i * xs + e]), i);
    const double2 o0 = to_d2(y0[e]);
    const double vr = f0 * o0.x - ar, vi = f0 * o0.y - ai;
    y0[e] = from_d2<T>(make_double2(vr, vi));
    if (y1) {
      const double2 o1 = to_d2(y1[e]);
      y1[e] = from_d2<T>(make_double2(f1 * o1.x - br - (gg.x * vr - gg.y * vi), f1 * o1.y - bi - (gg.x * vi + gg.y * vr)));
    }
  }
}

template <typename T>
void launch_mlincomb2(cplx<T>* Y0, long yk0, cplx<T>* Y1, long yk1, const cplx<T>* X, long xk, long xi, int J,
                      const double2* c, int ldc, int nk, long n, const int* act, hipStream_t s) {
  if (nk <= 0) return;
  long nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  if ((double)J * xi + n < 4294967296.0)
    BW_LAUNCH("k_mlincomb2", active_units(act, nk, J, s), (k_mlincomb2<T, uint32_t>), dim3((unsigned)nb, 1, nk),
              dim3(256), 0, s, Y0, yk0, Y1, yk1, X, xk, xi, J, c, ldc, n, act);
  else
    BW_LAUNCH("k_mlincomb2", active_units(act, nk, J, s), (k_mlincomb2<T, size_t>), dim3((unsigned)nb, 1, nk),
              dim3(256), 0, s, Y0, yk0, Y1, yk1, X, xk, xi, J, c, ldc, n, act);
}

template <typename T>
__global__ void k_scale_copy(const cplx<T>* __restrict__ X, long xk, cplx<T>* __restrict__ Y, long yk,
                             const double* __restrict__ sc, long n, const int* act) {
  const int k = blockIdx.y;
  if (act && !act[k]) return;
  const double f = sc[k];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double2 a = to_d2(X[(size_t)k * xk + e]);
    Y[(size_t)k * yk + e] = from_d2<T>(make_double2(a.x * f, a.y * f));
  }
}

template <typename T>
void launch_scale_copy(const cplx<T>* X, long xk, cplx<T>* Y, long yk, const double* sc, int nk, long n,
                       const int* act, hipStream_t s) {
  if (nk <= 0) return;
  long nb = (n + 255) / 256;
  if (nb > 512) nb = 512;
  hipLaunchKernelGGL((k_scale_copy<T>), dim3((unsigned)nb, nk), dim3(256), 0, s, X, xk, Y, yk, sc, n, act);
}

template <typename T>
__global__ void k_set_entries(cplx<T>* U, long vstride, long nvox, int nent, const long* vec, const long* vox,
                              const double* val, int add) {
  const int t = threadIdx.x;
  if (t >= nent * 3) return;
  const int e = t / 3, c = t - 3 * e;
  cplx<T>& u = U[(size_t)vec[e] * vstride + (size_t)c * nvox + vox[e]];
  if (add)
    u.x = (T)((double)u.x + val[t]);
  else
    u = from_d2<T>(make_double2(val[t], 0.0));
}

template <typename T>
void launch_set_entries(cplx<T>* U, long vstride, long nvox, int nent, const long* vec, const long* vox,
                        const double* val, hipStream_t s, bool add) {
  BW_REQUIRE(nent * 3 <= 256, BW_EINVAL, "too many entries");
  hipLaunchKernelGGL((k_set_entries<T>), dim3(1), dim3(256), 0, s, U, vstride, nvox, nent, vec, vox, val,
                     (int)add);
}

// X_p[e] += amp * (u1 + i u2) with u1, u2 uniform in [-1, 1) from a 64-bit
// counter hash (splitmix64 finalizer) of (seed, p, e): a deterministic
// pseudo-random perturbation, identical for every launch configuration.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
template <typename T>
__global__ void k_add_hash(cplx<T>* X, long n, long vstride, int nv, unsigned long long seed, double amp) {
  const long total = (long)nv * n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long p = e / n, i = e - p * n;
    const unsigned long long h = mix64(seed + 0x9e3779b97f4a7c15ULL * (unsigned long long)(p * n + i + 1));
    const double u1 = (double)(h >> 40) * (2.0 / 16777216.0) - 1.0;
    const double u2 = (double)((h >> 16) & 0xffffffULL) * (2.0 / 16777216.0) - 1.0;
    cplx<T>& x = X[p * vstride + i];
    x.x = (T)((double)x.x + amp * u1);
    x.y = (T)((double)x.y + amp * u2);
  }
}
template <typename T>
void launch_add_hash(cplx<T>* X, long n, long vstride, int nv, unsigned long long seed, double amp, hipStream_t s) {
  const long total = (long)nv * n;
  if (total == 0) return;
  long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((k_add_hash<T>), dim3((unsigned)blocks), dim3(256), 0, s, X, n, vstride, nv, seed, amp);
}

#define BW_INST_BLOCK(T)                                                                                          \
  template void launch_gram<T>(const cplx<T>*, int, const cplx<T>*, int, long, long, double2*, DevBuf&,            \
                               unsigned*, hipStream_t);                                                                      \
  template void launch_ritz<T>(const cplx<T>*, int, const double2*, int, cplx<T>*, int, long, long, hipStream_t,   \
                               bool);                                                                              \
  template void launch_dots<T>(const cplx<T>*, const cplx<T>*, int, long, long, double2*, DevBuf&, unsigned*,     \
                               hipStream_t);                                                                      \
  template void launch_lincomb<T>(const cplx<T>*, const cplx<T>*, const double*, cplx<T>*, int, long, long,       \
                                  hipStream_t);                                                                   \
  template void launch_scale_cols<T>(const cplx<T>*, const double*, cplx<T>*, int, long, long, hipStream_t);      \
  template void launch_deflate<T>(cplx<T>*, cplx<T>*, const cplx<T>*, int, long, long, double2*, hipStream_t);    \
  template void launch_planewaves<T>(cplx<T>*, int, long, const long*, const double*, hipStream_t);             \
  template void launch_mdot2<T>(const cplx<T>*, long, long, int, const cplx<T>*, long, const cplx<T>*, long, int,  \
                                long, const int*, double2*, double2*, int, DevBuf&, hipStream_t);                   \
  template void launch_mlincomb2<T>(cplx<T>*, long, cplx<T>*, long, const cplx<T>*, long, long, int,              \
                                    const double2*, int, int, long, const int*, hipStream_t);                      \
  template void launch_scale_copy<T>(const cplx<T>*, long, cplx<T>*, long, const double*, int, long, const int*,  \
                                     hipStream_t);                                                                \
  template void launch_set_entries<T>(cplx<T>*, long, long, int, const long*, const long*, const double*,        \
                                      hipStream_t, bool);                                                         \
  template void launch_add_hash<T>(cplx<T>*, long, long, int, unsigned long long, double, hipStream_t);

BW_INST_BLOCK(double)
BW_INST_BLOCK(float)
template void launch_convert<float, double>(const cplx<float>*, cplx<double>*, size_t, hipStream_t);
template void launch_convert<double, float>(const cplx<double>*, cplx<float>*, size_t, hipStream_t);

}  // namespace bw
