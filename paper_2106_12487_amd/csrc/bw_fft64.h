// Length-64 transforms held in registers: the passes of the K operator for
// axes of 64 points (8 x 8 decomposition, one LDS exchange per transform).
//
// Eight threads share a line.  Thread j (0..7) loads the points x[j + 8 r],
// r < 8, straight from global memory, runs the first radix-8 stage in
// registers (its outputs are the Stockham indices 8 j + r), swaps through LDS
// to the second stage's inputs j + 8 r, applies the twiddles w^(r j)
// (w = e^{-+2 pi i / 64}) and runs the second radix-8 stage; it then holds
// X[j + 8 r], the same index set it loaded, so pointwise work between an
// inverse and a forward transform needs no further exchange.  Per transform
// that is one LDS write and one read of the tile, against a load stage, two
// in-place passes and a read-back for the generic LDS FFT.  Consecutive
// transforms alternate between two LDS buffers so that each needs a single
// barrier.
#pragma once
// Included by bw_ops_impl.h after the generic kernels and before the launchers.

namespace bw {

template <typename T>
__device__ __forceinline__ void load_tw64(cplx<T> (&w)[8], const cplx<T>* __restrict__ tw, int j) {
#pragma unroll
  for (int r = 0; r < 8; ++r) w[r] = tw[r * j];
}

// v: x[j + 8 r] in, X[j + 8 r] out; slot(n) is the LDS position of index n of
// this thread's line.  Ends without a barrier: the next call must use the
// other buffer (or the caller synchronizes).
template <typename T, bool INV, class Slot>
__device__ __forceinline__ void fft64_regs(cplx<T> (&v)[8], cplx<T>* buf, const Slot& slot, int j,
                                           const cplx<T> (&w)[8]) {
  using V = cplx<T>;
  SmallDFT<8, INV, V>::run(v);
#pragma unroll
  for (int r = 0; r < 8; ++r) buf[slot(8 * j + r)] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = buf[slot(j + 8 * r)];
#pragma unroll
  for (int r = 1; r < 8; ++r) v[r] = INV ? cmulc(v[r], w[r]) : cmul(v[r], w[r]);
  SmallDFT<8, INV, V>::run(v);
}

// Row tiles (axis 2, contiguous): 32 rows per block, lane = 8 * row + j so
// that eight neighbouring lanes read 64 contiguous bytes of a row.  LDS row
// pitch 72 with a skew of one slot per 8 to spread the banks.
constexpr int R64_ROWS = 32;
constexpr int R64_PITCH = 72;
struct RowSlot {
  int base;
  __device__ __forceinline__ int operator()(int n) const { return base + n + (n >> 3); }
};
// Column tiles (axes 0 and 1): 32 consecutive lines, lane = line + 32 j.
constexpr int C64_LINES = 32;
struct ColSlot {
  int line;
  __device__ __forceinline__ int operator()(int n) const { return n * C64_LINES + line; }
};

// ---------------------------------------------------------------------------
// K, first pass for n2 = 64 (same contract as k_strain_row)
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_strain_row64(const cplx<T>* __restrict__ U, cplx<T>* __restrict__ Pp,
                                                     cplx<T>* __restrict__ W, const double* __restrict__ qtab,
                                                     int n0, int n1, long nvox, int tpv,
                                                     const cplx<T>* __restrict__ tw, const int* __restrict__ active,
                                                     const double* __restrict__ beta, C21v<T> C0) {
  using V = cplx<T>;
  __shared__ V lds[2][R64_ROWS * R64_PITCH];
  const int v = blockIdx.x / tpv;
  const int tile = blockIdx.x - v * tpv;
  if (active && !active[v]) return;
  const int tid = threadIdx.x;
  const int j = tid & 7, line = tid >> 3;
  const int row = tile * R64_ROWS + line;
  const int i0 = row / n1, i1 = row - i0 * n1;
  const double* q = qtab + (size_t)v * (n0 + n1 + 64);
  const T qa = (T)q[i0], qb = (T)q[n0 + i1];
  T qc[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) qc[r] = (T)q[n0 + n1 + j + 8 * r];
  V w[8];
  load_tw64<T>(w, tw, j);
  const size_t rbase = (size_t)row * 64 + j;
  V u[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 8; ++r) u[c][r] = U[((size_t)v * 3 + c) * nvox + rbase + 8 * r];
  if (MODE == 1) {
    const T bt = (T)beta[v];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      V in[3] = {u[0][r], u[1][r], u[2][r]}, z[3];
      precond3<T, V>(C0, qa, qb, qc[r], in, z);
      if (bt != T(0)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) z[c] = caxpy(z[c], bt, Pp[((size_t)v * 3 + c) * nvox + rbase + 8 * r]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Pp[((size_t)v * 3 + c) * nvox + rbase + 8 * r] = z[c];
        u[c][r] = z[c];
      }
    }
  }
  const RowSlot slot{line * R64_PITCH};
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    V e[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      switch (c) {
        case 0: e[r] = cscale(u[0][r], qa); break;
        case 1: e[r] = cscale(u[1][r], qb); break;
        case 2: e[r] = cscale(u[2][r], qc[r]); break;
        case 3: e[r] = cadd(cscale(u[1][r], qc[r]), cscale(u[2][r], qb)); break;
        case 4: e[r] = cadd(cscale(u[0][r], qc[r]), cscale(u[2][r], qa)); break;
        default: e[r] = cadd(cscale(u[0][r], qb), cscale(u[1][r], qa)); break;
      }
    }
    fft64_regs<T, true>(e, lds[c & 1], slot, j, w);
#pragma unroll
    for (int r = 0; r < 8; ++r) W[((size_t)v * 6 + c) * nvox + rbase + 8 * r] = e[r];
  }
}

// ---------------------------------------------------------------------------
// K, last pass for n2 = 64 (same contract as k_row_div; partials per tile)
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_row_div64(const cplx<T>* __restrict__ W, cplx<T>* __restrict__ Y,
                                                  const double* __restrict__ qtab, int n0, int n1, long nvox,
                                                  int tpv, const cplx<T>* __restrict__ tw,
                                                  const int* __restrict__ active, const cplx<T>* __restrict__ Pp,
                                                  PcgDev pd, T oscale) {
  using V = cplx<T>;
  __shared__ V lds[2][R64_ROWS * R64_PITCH];
  __shared__ double sh[NT / 64];
  const int v = blockIdx.x / tpv;
  const int tile = blockIdx.x - v * tpv;
  if (active && !active[v]) return;
  const int tid = threadIdx.x;
  const int j = tid & 7, line = tid >> 3;
  const int row = tile * R64_ROWS + line;
  const int i0 = row / n1, i1 = row - i0 * n1;
  const double* q = qtab + (size_t)v * (n0 + n1 + 64);
  const T qa = (T)q[i0], qb = (T)q[n0 + i1];
  T qc[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) qc[r] = (T)q[n0 + n1 + j + 8 * r];
  V w[8];
  load_tw64<T>(w, tw, j);
  const size_t rbase = (size_t)row * 64 + j;
  const RowSlot slot{line * R64_PITCH};
  V acc[3][8];
#pragma unroll
  for (int r = 0; r < 8; ++r) acc[0][r] = acc[1][r] = acc[2][r] = V{0, 0};
  V nxt[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) nxt[r] = W[((size_t)v * 6) * nvox + rbase + 8 * r];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    V e[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) e[r] = nxt[r];
    if (c < 5) {
#pragma unroll
      for (int r = 0; r < 8; ++r) nxt[r] = W[((size_t)v * 6 + c + 1) * nvox + rbase + 8 * r];
    }
    fft64_regs<T, false>(e, lds[c & 1], slot, j, w);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      switch (c) {
        case 0: acc[0][r] = caxpy(acc[0][r], qa, e[r]); break;
        case 1: acc[1][r] = caxpy(acc[1][r], qb, e[r]); break;
        case 2: acc[2][r] = caxpy(acc[2][r], qc[r], e[r]); break;
        case 3: acc[1][r] = caxpy(acc[1][r], qc[r], e[r]); acc[2][r] = caxpy(acc[2][r], qb, e[r]); break;
        case 4: acc[0][r] = caxpy(acc[0][r], qc[r], e[r]); acc[2][r] = caxpy(acc[2][r], qa, e[r]); break;
        default: acc[0][r] = caxpy(acc[0][r], qb, e[r]); acc[1][r] = caxpy(acc[1][r], qa, e[r]); break;
      }
    }
  }
  double part = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const V o = cscale(acc[c][r], oscale);
      Y[((size_t)v * 3 + c) * nvox + rbase + 8 * r] = o;
      if (MODE == 1) {
        const V pv = Pp[((size_t)v * 3 + c) * nvox + rbase + 8 * r];
        part += (double)pv.x * (double)o.x + (double)pv.y * (double)o.y;
      }
    }
  if (MODE == 1) {
    const double vals[1] = {part};
    store_partials<1>(vals, pd.partial, v, tile, pd.max_blocks, sh);
  }
}

// ---------------------------------------------------------------------------
// FFT along axis 1 for n1 = 64 (stride n2, n2 % 32 == 0), in place; lines are
// (plane, column) with plane = (component, i0).  tpv = planes * n2 / 32.
// ---------------------------------------------------------------------------
template <typename T, bool INV, int PCG = 0>
__global__ __launch_bounds__(NT) void k_axis1_64(cplx<T>* __restrict__ X, int n2, long vec_stride, int tpv,
                                                 const cplx<T>* __restrict__ tw, const int* __restrict__ active) {
  using V = cplx<T>;
  __shared__ V lds[64 * C64_LINES];
  const int v = blockIdx.x / tpv;
  if (active && !active[v]) return;
  const int tile = blockIdx.x - v * tpv;
  const int tid = threadIdx.x;
  const int line = tid & (C64_LINES - 1), j = tid >> 5;
  const int tpp = n2 / C64_LINES;
  const int plane = tile / tpp;
  const int col = (tile - plane * tpp) * C64_LINES + line;
  V* base = X + (size_t)v * vec_stride + (size_t)plane * 64 * n2 + col + (size_t)j * n2;
  V w[8];
  load_tw64<T>(w, tw, j);
  V e[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) e[r] = base[(size_t)8 * r * n2];
  fft64_regs<T, INV>(e, lds, ColSlot{line}, j, w);
#pragma unroll
  for (int r = 0; r < 8; ++r) base[(size_t)8 * r * n2] = e[r];
}

// ---------------------------------------------------------------------------
// Axis 0 for n0 = 64 (same contract as k_axis0_op; n12 % 32 == 0): inverse
// FFT, stiffness contraction (OP 0) or density scaling (OP 1), forward FFT.
// ---------------------------------------------------------------------------
template <typename T, int OP, int PCG = 0>
__global__ __launch_bounds__(NT, 2) void k_axis0_op64(cplx<T>* __restrict__ X, long n12, long nvox, int tpv,
                                                   const uint16_t* __restrict__ gmap, const T* __restrict__ Ctab,
                                                   T scale, const cplx<T>* __restrict__ tw,
                                                   const int* __restrict__ active) {
  using V = cplx<T>;
  constexpr int NC = OP == 0 ? 6 : 3;
  __shared__ V lds[2][64 * C64_LINES];
  const int v = blockIdx.x / tpv;
  if (active && !active[v]) return;
  const int tile = blockIdx.x - v * tpv;
  const int tid = threadIdx.x;
  const int line = tid & (C64_LINES - 1), j = tid >> 5;
  const long pos = (long)tile * C64_LINES + line;
  V w[8];
  load_tw64<T>(w, tw, j);
  // 32-bit offsets within the vector (NC * nvox < 2^31, checked by the host)
  cplx<T>* Xv = X + (size_t)v * NC * nvox;
  const int o0 = (int)pos + j * (int)n12, s8 = 8 * (int)n12, cs = (int)nvox;
  V x[NC][8];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < 8; ++r) x[c][r] = Xv[c * cs + o0 + r * s8];
  const ColSlot slot{line};
#pragma unroll
  for (int c = 0; c < NC; ++c) fft64_regs<T, true>(x[c], lds[c & 1], slot, j, w);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int g = gmap[o0 + r * s8];
    if (OP == 0) {
      T cg[21];
#pragma unroll
      for (int i = 0; i < 21; ++i) cg[i] = Ctab[g * 21 + i];
      V e[6], sg[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = x[c][r];
      contract6<T, V>(cg, e, sg, scale);
#pragma unroll
      for (int c = 0; c < 6; ++c) x[c][r] = sg[c];
    } else {
      const T rs = Ctab[g] * scale;
#pragma unroll
      for (int c = 0; c < NC; ++c) x[c][r] = cscale(x[c][r], rs);
    }
    // keep the table loads of one point at a time in flight (register pressure)
    asm volatile("" ::: "memory");
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    fft64_regs<T, false>(x[c], lds[(NC + c) & 1], slot, j, w);
#pragma unroll
    for (int r = 0; r < 8; ++r) Xv[c * cs + o0 + r * s8] = x[c][r];
  }
}

}  // namespace bw
