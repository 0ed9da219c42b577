// Slab passes of the K operator for FP32 cells with n1 = n2 = 128: the
// transforms along axes 2 and 1 of one (vector, i0) slab, a 128 x 128 plane of
// one component, run in one workgroup with the plane staged in LDS, so that K
// takes three passes over HBM (Sec. 3.2 eq. hatA):
//
//   k_slab_strain  strain e^ = B(q) u^ and the inverse 2D FFT over (i1, i2)
//                  of each of its six components (reads 3, writes 6 words)
//   k_axis0_op_r   inverse FFT along axis 0, s = C(x) e, forward FFT along
//                  axis 0 (reads and writes 6 words, reads the grain index)
//   k_slab_div     forward 2D FFT over (i1, i2) of the six stress components
//                  and the divergence B(q)^T s^ (reads 6, writes 3 words)
//
// A workgroup of 1024 threads takes a slab (one per CU: the plane fills the
// LDS); thread t handles line a = t >> 3 with lane j = t & 7 in both phases of
// a 2D transform: 16 points n = j + 8 m (m < 16) of row a (along i2), then of
// column a (along i1).  A 128-point transform is a 16-point DFT over m in
// registers, the twiddles w^(j k1), one exchange among the line's 8 lanes (one
// wavefront, in the line's own LDS region), and 8-point DFTs over j: lane j
// ends with X[2 j + p + 16 k2], p < 2, k2 < 8.  Rows are written to the LDS
// plane at those positions and read back as columns; a component costs two
// workgroup barriers.
//
// LDS: line l owns slots [136 l, 136 l + 136) (a pitch of 8 mod 16 slots puts
// neighbouring lines in opposite halves of the 32 banks).  The exchange puts
// (k1, j) at slot 8 k1 + (j ^ (k1 >> 1)); the plane puts column k of row l at
// slot k ^ (l & 7); lane j's twiddles start at slot 17 j of their own table.
// Every access pattern (exchange writes and reads, row writes, column reads,
// twiddle reads) then spreads each group of 16 lanes of an 8-byte access
// over all 32 banks (and each group of 32 lanes over 64), and every address is
// a per-thread base plus a constant.
// Global accesses are a uniform base plus a 32-bit lane offset and a constant.
// Keeping addresses that cheap is what leaves the registers for three live
// 16-point sets per thread (at most 128 registers per lane at 1024 threads).
//
// The sources of the strain components are held one at a time in registers
// (in the order u0, u2, u1, u2), so u2 is read twice per slab, and the next
// source is loaded while the current component is transformed; the divergence
// accumulates two output components at a time, so each stress component is
// read once.  In PCG mode the strain pass forms the direction p = z + beta p
// from z = P^ r, which the update kernel left in the K p buffer.
#pragma once
// Included by bw_ops_impl.h after bw_fftreg.h.

namespace bw {

constexpr int SLAB_NT = 1024;
constexpr int SLAB_N = 128;
constexpr int SLAB_LP = 136;                // LDS slots per line region
constexpr int SLAB_LDS = SLAB_N * SLAB_LP;
constexpr int SLAB_TWP = 17;                // twiddle table pitch per lane (slots)

// exp(2 pi i e / 16) for e < 16 (cosine and sine)
__device__ __forceinline__ float2 w16(int e, bool inv) {
  constexpr float c[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                           0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                           -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                           0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
  const float cc = c[e & 15], ss = c[(e + 12) & 15];   // sin(x) = cos(x - pi/2)
  return float2{cc, inv ? ss : -ss};
}

// 16-point DFT in registers, natural order in and out: x_k = sum_m x_m w^(s m k)
// (s = +1 inverse, -1 forward), as 4 x 4 with the twiddles w16^(m1 k'), in place
// (the last step's transposition is a renaming of registers).
template <bool INV> __device__ __forceinline__ void dft16(float2 (&x)[16]) {
#pragma unroll
  for (int m1 = 0; m1 < 4; ++m1) {
    float2 t[4] = {x[m1], x[m1 + 4], x[m1 + 8], x[m1 + 12]};
    SmallDFT<4, INV, float2>::run(t);
#pragma unroll
    for (int k = 0; k < 4; ++k) x[m1 + 4 * k] = (m1 * k == 0) ? t[k] : cmul(t[k], w16(m1 * k, INV));
  }
  float2 y[16];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float2 t[4] = {x[4 * k], x[4 * k + 1], x[4 * k + 2], x[4 * k + 3]};
    SmallDFT<4, INV, float2>::run(t);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) y[k + 4 * k2] = t[k2];
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = y[i];
}

// The 128-point transform of the line whose LDS region starts at `reg`, held by
// its 8 lanes (lane j).  On entry x[m] = x_(j + 8 m); on exit x[p * 8 + k2] =
// X_(2 j + p + 16 k2).  tw: the LDS table tw[j * 17 + k1] = exp(-2 pi i j k1 /
// 128) (a pitch of 17 slots: with 16, the 8 lanes of a line, reading the same
// k1, would all hit one bank pair).  The exchange is wavefront-local (the line's lanes are 8 consecutive
// lanes of one wavefront).
template <bool INV>
__device__ __forceinline__ void slab_fft128(float2 (&x)[16], float2* reg, int j, const float2* tw) {
  dft16<INV>(x);
  const float2* twj = tw + j * SLAB_TWP;
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) x[k1] = INV ? cmulc(x[k1], twj[k1]) : cmul(x[k1], twj[k1]);
  xsync<true>();
#pragma unroll
  for (int c = 0; c < 8; ++c) {              // (k1, j) at 8 k1 + (j ^ c), c = k1 >> 1
    float2* b = reg + (j ^ c);
    b[16 * c] = x[2 * c];
    b[16 * c + 8] = x[2 * c + 1];
  }
  xsync<true>();
  const float2* r = reg + 16 * j;            // rows k1 = 2 j + p
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    const float2* b = r + (jj ^ j);
    x[jj] = b[0];
    x[8 + jj] = b[8];
  }
  xsync<true>();
  SmallDFT<8, INV, float2>::run(&x[0]);
  SmallDFT<8, INV, float2>::run(&x[8]);
}

// output row (i1) of register i = p * 8 + k2 after a 2D transform, for lane j
__device__ __forceinline__ int slab_row(int j, int i) { return 2 * j + (i >> 3) + 16 * (i & 7); }

// 2D transform of one slab component: on entry thread (a, j) holds row a,
// points j + 8 m (i2); on exit column a (i2 = a), rows slab_row(j, i) (i1) in
// x[i].  Ends with the column exchange; the next call may start at once (the
// regions touched in between belong to the same lanes).
template <bool INV>
__device__ __forceinline__ void slab_fft2d(float2 (&x)[16], float2* S, const float2* tw, int a, int j) {
  // the lane's position, opaque to the compiler: the LDS addresses below are
  // recomputed for every component instead of being hoisted out of the
  // unrolled sequence, where they would hold many registers
  asm volatile("" : "+v"(a), "+v"(j));
  float2* reg = S + a * SLAB_LP;
  slab_fft128<INV>(x, reg, j, tw);            // rows (axis 2)
  {
    // column k = 2 j + p + 16 k2 of row a at slot k ^ (a & 7) = ((2 j + p) ^ (a & 7)) + 16 k2
    const int sw = a & 7;
    float2* b0 = reg + ((2 * j) ^ sw);       // p = 0
    float2* b1 = reg + ((2 * j + 1) ^ sw);   // p = 1
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
      b0[16 * k2] = x[k2];
      b1[16 * k2] = x[8 + k2];
    }
  }
  __syncthreads();
  {
    // rows j + 8 m, column a at slot a ^ (row & 7) = a ^ j
    const float2* b = S + j * SLAB_LP + (a ^ j);
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = b[m * 8 * SLAB_LP];
  }
  __syncthreads();                            // every column read before the column exchanges write
  slab_fft128<INV>(x, reg, j, tw);            // columns (axis 1)
}

// LDS tables of a slab workgroup: the twiddles per lane and, as floats, the
// shifted wave numbers of axes 1 and 2 of vector v (visible after a barrier).
__device__ __forceinline__ void slab_tables(float2* tw, float* q1, float* q2, const float2* __restrict__ twg,
                                            const double* __restrict__ q, int n0, int t) {
  if (t < 128) tw[(t >> 4) * SLAB_TWP + (t & 15)] = twg[(t >> 4) * (t & 15)];
  else if (t < 256) q1[t - 128] = (float)q[n0 + t - 128];
  else if (t < 384) q2[t - 256] = (float)q[n0 + SLAB_N + t - 256];
}

// element `off` (float2 units, 32-bit) of a uniform base
__device__ __forceinline__ const float2& at(const float2* base, uint32_t off) { return base[off]; }

// ---------------------------------------------------------------------------
// Pass 1: strain and inverse 2D FFT.  Grid: nvec * n0 workgroups of 1024.
// MODE 0: u = U.  MODE 1: U holds z = P^ r and Pp the direction p, updated
// here to p = z + beta p (p = z where beta = 0), and u = p.
// W: [vec][6][n0][128][128], real space along i1, i2.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(SLAB_NT, 1) void k_slab_strain(const float2* __restrict__ U, float2* __restrict__ Pp,
                                                           float2* __restrict__ W, const double* __restrict__ qtab,
                                                           int n0, long nvox, const float2* __restrict__ twg,
                                                           const int* __restrict__ active,
                                                           const double* __restrict__ beta) {
  __shared__ float2 S[SLAB_LDS];
  __shared__ float2 tw[8 * SLAB_TWP];
  __shared__ float q1s[SLAB_N], q2s[SLAB_N];
  const int v = blockIdx.x / n0;
  const int i0 = blockIdx.x - v * n0;
  if (active && !active[v]) return;
  const int t = threadIdx.x, a = t >> 3, j = t & 7;
  const double* q = qtab + (size_t)v * (n0 + 2 * SLAB_N);
  slab_tables(tw, q1s, q2s, twg, q, n0, t);
  const float qa = (float)q[i0], qb = (float)q[n0 + a];
  const float* qc = q2s + j;                  // qc[8 m] = q_2(j + 8 m)
  const float bt = MODE == 1 ? (float)beta[v] : 0.0f;
  const size_t slab = (size_t)i0 * SLAB_N * SLAB_N;
  const uint32_t cs = (uint32_t)nvox;         // component stride (6 nvox < 2^31)
  const float2* Uv = U + (size_t)v * 3 * nvox + slab;
  float2* Pv = MODE == 1 ? Pp + (size_t)v * 3 * nvox + slab : nullptr;
  float2* Wv = W + (size_t)v * 6 * nvox + slab;
  const uint32_t lo = (uint32_t)(a * SLAB_N + j);   // row a, point j (+ 8 m)
  float2 s[16], e[16], f[16];
  auto fetch = [&](int c) {                   // raw loads of component c (MODE 1: z)
    // MODE 0 reads only the input, whose loads could otherwise be hoisted above
    // the work before them (while f is still live there)
    if (MODE == 0) asm volatile("" ::: "memory");
    const float2* b = Uv + (size_t)c * cs;
#pragma unroll
    for (int m = 0; m < 16; ++m) f[m] = at(b, lo + 8 * m);
  };
  // MODE 1: the previous direction of component c, loaded into e while e is
  // free (no fourth set of registers for it)
  auto load_p = [&](int c) {
    if (MODE == 1 && bt != 0.0f) {
      const float2* b = Pv + (size_t)c * cs;
#pragma unroll
      for (int m = 0; m < 16; ++m) e[m] = at(b, lo + 8 * m);
    }
  };
  // the values of component c at its first use: MODE 1 forms and stores the new
  // direction from the fetched z and the previous direction in e[m] (read before
  // the caller overwrites e[m])
  auto source = [&](int c, int m) -> float2 {
    float2 u = f[m];
    if (MODE == 1) {
      if (bt != 0.0f) u = caxpy(u, bt, e[m]);
      float2* b = Pv + (size_t)c * cs;
      b[lo + 8 * m] = u;
    }
    return u;
  };
  auto finish = [&](int c) {
    slab_fft2d<true>(e, S, tw, a, j);
    int aa = a, jj = j;
    asm volatile("" : "+v"(aa), "+v"(jj));
    float2* b = Wv + (size_t)c * cs;
    const uint32_t o = (uint32_t)(2 * jj * SLAB_N + aa);
#pragma unroll
    for (int i = 0; i < 16; ++i) b[o + (uint32_t)((i >> 3) + 16 * (i & 7)) * SLAB_N] = e[i];
  };
  __syncthreads();                            // tables
  fetch(0);
  load_p(0);
#pragma unroll
  for (int m = 0; m < 16; ++m) s[m] = source(0, m);
  fetch(2);                                   // u2, in flight during the first transform
  // e0 = qa u0
#pragma unroll
  for (int m = 0; m < 16; ++m) e[m] = cscale(s[m], qa);
  finish(0);
  // e4 = qc u0 + qa u2
  load_p(2);
#pragma unroll
  for (int m = 0; m < 16; ++m) e[m] = caxpy(cscale(s[m], qc[8 * m]), qa, source(2, m));
  fetch(1);
  finish(4);
  // e5 = qb u0 + qa u1; then hold u1
  load_p(1);
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const float2 u1 = source(1, m);
    e[m] = caxpy(cscale(s[m], qb), qa, u1);
    s[m] = u1;
  }
  // u2 again: the direction stored above by this thread (MODE 1) or the input
  if (MODE == 1) {
    const float2* b = Pv + (size_t)2 * cs;
#pragma unroll
    for (int m = 0; m < 16; ++m) f[m] = at(b, lo + 8 * m);
  } else {
    fetch(2);
  }
  finish(5);
  // e1 = qb u1
#pragma unroll
  for (int m = 0; m < 16; ++m) e[m] = cscale(s[m], qb);
  finish(1);
  // e3 = qc u1 + qb u2; then hold u2
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    e[m] = caxpy(cscale(s[m], qc[8 * m]), qb, f[m]);
    s[m] = f[m];
  }
  finish(3);
  // e2 = qc u2
#pragma unroll
  for (int m = 0; m < 16; ++m) e[m] = cscale(s[m], qc[8 * m]);
  finish(2);
}

// ---------------------------------------------------------------------------
// Pass 3: forward 2D FFT of the stress and divergence out_i = q_j s^_ij, scaled
// by oscale.  MODE 1 also writes this slab's partial <p, K p> (FP64) as block
// i0 of vector v.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(SLAB_NT, 1) void k_slab_div(const float2* __restrict__ W, float2* __restrict__ Y,
                                                        const double* __restrict__ qtab, int n0, long nvox,
                                                        const float2* __restrict__ twg,
                                                        const int* __restrict__ active,
                                                        const float2* __restrict__ Pp, PcgDev pd, float oscale) {
  __shared__ float2 S[SLAB_LDS];
  __shared__ float2 tw[8 * SLAB_TWP];
  __shared__ float q1s[SLAB_N], q2s[SLAB_N];
  __shared__ double red[SLAB_NT / 64];
  const int v = blockIdx.x / n0;
  const int i0 = blockIdx.x - v * n0;
  if (active && !active[v]) return;
  const int t = threadIdx.x, a = t >> 3, j = t & 7;
  const double* q = qtab + (size_t)v * (n0 + 2 * SLAB_N);
  slab_tables(tw, q1s, q2s, twg, q, n0, t);
  const float qa = (float)q[i0], qc = (float)q[n0 + SLAB_N + a];
  const size_t slab = (size_t)i0 * SLAB_N * SLAB_N;
  const uint32_t cs = (uint32_t)nvox;
  const float2* Wv = W + (size_t)v * 6 * nvox + slab;
  float2* Yv = Y + (size_t)v * 3 * nvox + slab;
  const float2* Pv = MODE == 1 ? Pp + (size_t)v * 3 * nvox + slab : nullptr;
  const uint32_t lo = (uint32_t)(a * SLAB_N + j);     // row a, point j (+ 8 m)
  const float* qbj = q1s + 2 * j;                      // q_1 of row 2 j + p + 16 k2
  double part = 0.0;
  auto QB = [&](int i) { return qbj[(i >> 3) + 16 * (i & 7)]; };
  auto load = [&](float2 (&x)[16], int c) {
    // the loads of a component are not hoisted above the previous one's work
    __builtin_amdgcn_sched_barrier(0);
    const float2* b = Wv + (size_t)c * cs;
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = at(b, lo + 8 * m);
    slab_fft2d<false>(x, S, tw, a, j);
  };
  auto store = [&](const float2 (&o)[16], int c) {
    __builtin_amdgcn_sched_barrier(0);
    int aa = a, jj = j;
    asm volatile("" : "+v"(aa), "+v"(jj));
    float2* b = Yv + (size_t)c * cs;
    const float2* pb = MODE == 1 ? Pv + (size_t)c * cs : nullptr;
    const uint32_t o0 = (uint32_t)(2 * jj * SLAB_N + aa);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t off = o0 + (uint32_t)((i >> 3) + 16 * (i & 7)) * SLAB_N;
      const float2 ov = cscale(o[i], oscale);
      b[off] = ov;
      if (MODE == 1) {
        const float2 pv = at(pb, off);
        part += (double)pv.x * (double)ov.x + (double)pv.y * (double)ov.y;
        // the direction's loads four at a time (registers: three 16-point sets
        // are live here)
        if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  __syncthreads();                            // tables
  float2 A[16], B[16], T[16];
  // s5 (sigma_12): out0 += qb s5, out1 += qa s5
  load(T, 5);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    A[i] = cscale(T[i], QB(i));
    B[i] = cscale(T[i], qa);
  }
  // s0: out0 += qa s0
  load(T, 0);
#pragma unroll
  for (int i = 0; i < 16; ++i) A[i] = caxpy(A[i], qa, T[i]);
  // s1: out1 += qb s1
  load(T, 1);
#pragma unroll
  for (int i = 0; i < 16; ++i) B[i] = caxpy(B[i], QB(i), T[i]);
  // s4 (sigma_13): out0 += qc s4 (complete), out2 = qa s4
  load(T, 4);
#pragma unroll
  for (int i = 0; i < 16; ++i) A[i] = caxpy(A[i], qc, T[i]);
  store(A, 0);
#pragma unroll
  for (int i = 0; i < 16; ++i) A[i] = cscale(T[i], qa);
  // s3 (sigma_23): out1 += qc s3 (complete), out2 += qb s3
  load(T, 3);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    B[i] = caxpy(B[i], qc, T[i]);
    A[i] = caxpy(A[i], QB(i), T[i]);
  }
  store(B, 1);
  // s2: out2 += qc s2 (complete)
  load(T, 2);
#pragma unroll
  for (int i = 0; i < 16; ++i) A[i] = caxpy(A[i], qc, T[i]);
  store(A, 2);
  if (MODE == 1) {
    double w = wave_sum(part);
    if ((t & 63) == 0) red[t >> 6] = w;
    __syncthreads();
    if (t == 0) {
      double sum = 0.0;
      for (int i = 0; i < SLAB_NT / 64; ++i) sum += red[i];
      pd.partial[(size_t)v * pd.max_blocks + i0] = sum;
    }
  }
}

}  // namespace bw
