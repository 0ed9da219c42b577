// Register-resident FFTs of power-of-two length N = 16 .. 256 for the passes
// of the K operator: 8 points per thread, N / 8 threads per line, Stockham
// radix passes in registers (radix 8 first, then 8, 4 or 2) with one LDS
// exchange between consecutive passes.
//
// Layouts.  Thread j of a line holds 8 points.  "Layout A" is the natural
// load order x[j + m N/8] (m < 8); a transform that starts from layout A
// (decimation in time, `fft_dit`) ends with the outputs in "layout B", the
// Stockham write positions of its last pass.  The same pass network run
// backwards with the same twiddles (decimation in frequency, `fft_dif`) takes
// layout B to layout A; since the DFT matrix is symmetric it computes the same
// transform.  Kernels load in layout A, store wherever the transform leaves
// the data, and the axis-0 pass (inverse transform, pointwise contraction,
// forward transform) returns to layout A without any extra exchange.
//
// LDS traffic per transform: one write and one read of the tile per pass
// after the first, against a load stage, one read-write per pass and a
// read-back for the generic LDS FFT.  Consecutive exchanges alternate between
// two buffers, so each needs a single barrier.
#pragma once
// Included by bw_ops_impl.h after the generic kernels and before the launchers.

namespace bw {

template <int N> struct RegFFT {
  static_assert(N == 16 || N == 32 || N == 64 || N == 128 || N == 256, "register FFT length");
  static constexpr int T = N / 8;          // threads per line
  static constexpr int LINES = NT / T;     // lines per 256-thread block
  static constexpr int P = (N <= 64) ? 2 : 3;
  static constexpr int radix(int p) {
    return p == 0 ? 8 : (N == 16 ? 2 : N == 32 ? 4 : N == 64 ? 8 : p == 1 ? 8 : (N == 128 ? 2 : 4));
  }
  static constexpr int ns(int p) { return p == 0 ? 1 : (p == 1 ? 8 : 64); }
  // butterfly b, element r of pass p
  __device__ static constexpr int rpos(int p, int b, int r) { return b + r * (N / radix(p)); }
  __device__ static constexpr int wpos(int p, int b, int r) {
    return (b / ns(p)) * ns(p) * radix(p) + (b % ns(p)) + r * ns(p);
  }
  __device__ static constexpr int texp(int p, int b, int r) {
    return ns(p) == 1 ? 0 : r * (b % ns(p)) * (N / (ns(p) * radix(p)));
  }
  // register m of thread j in pass p: butterfly and element
  __device__ static constexpr int bfly(int p, int j, int m) { return j * (8 / radix(p)) + m / radix(p); }
  __device__ static constexpr int elem(int p, int m) { return m % radix(p); }
  __device__ static constexpr int posA(int j, int m) { return j + m * T; }
  __device__ static constexpr int posB(int j, int m) {
    return wpos(P - 1, bfly(P - 1, j, m), elem(P - 1, m));
  }
  static constexpr int BUF = LINES * (N + N / 8);  // elements per exchange buffer (row pitch with skew)
  static constexpr int BUFC = LINES * N;           // column tiles (no skew)
  static constexpr int NBUF = P > 2 ? 2 : 1;       // a single transform with one exchange needs one buffer
};

// Twiddles of passes 1 .. P-1 for thread j: w[p - 1][m] = tw[texp].
template <typename T, int N>
__device__ __forceinline__ void load_twr(cplx<T> (&w)[RegFFT<N>::P - 1][8], const cplx<T>* __restrict__ tw, int j) {
  using F = RegFFT<N>;
#pragma unroll
  for (int p = 1; p < F::P; ++p)
#pragma unroll
    for (int m = 0; m < 8; ++m)
      w[p - 1][m] = F::elem(p, m) == 0 ? cplx<T>{1, 0} : tw[F::texp(p, F::bfly(p, j, m), F::elem(p, m))];
}

template <int R, bool INV, typename V> __device__ __forceinline__ void dft_groups(V (&v)[8]) {
#pragma unroll
  for (int t = 0; t < 8 / R; ++t) SmallDFT<R, INV, V>::run(&v[t * R]);
}

template <int N, int p, bool INV, typename V> __device__ __forceinline__ void dft_pass(V (&v)[8]) {
  constexpr int R = RegFFT<N>::radix(p);
  dft_groups<R, INV>(v);
}

// Synchronization of one exchange: the workgroup, or only the wavefront when
// every line of the tile lies inside one wavefront (N / 8 consecutive lanes
// with lane = (N / 8) line + j).  A wavefront's LDS operations execute in issue
// order; the wavefront-scope fences keep the compiler from moving accesses
// across the exchange.  Consecutive exchanges alternate between two buffers, so
// the writes of one exchange never overtake the reads of the previous one.
// The plane pass uses the wavefront form; the row passes keep the workgroup
// form, which measured faster there (the workgroup's stores stay together).
template <bool WAVE> __device__ __forceinline__ void xsync() {
  if (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Decimation in time: v holds layout A on entry, layout B on exit.
template <typename T, int N, bool INV, bool WAVE = false, class Slot>
__device__ __forceinline__ void fft_dit(cplx<T> (&v)[8], cplx<T>* buf0, cplx<T>* buf1, int& parity, const Slot& slot,
                                        int j, const cplx<T> (&w)[RegFFT<N>::P - 1][8]) {
  using F = RegFFT<N>;
  using V = cplx<T>;
  dft_pass<N, 0, INV>(v);
#pragma unroll
  for (int p = 1; p < F::P; ++p) {
    V* buf = (parity++ & 1) ? buf1 : buf0;
#pragma unroll
    for (int m = 0; m < 8; ++m) buf[slot(F::wpos(p - 1, F::bfly(p - 1, j, m), F::elem(p - 1, m)))] = v[m];
    xsync<WAVE>();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const V x = buf[slot(F::rpos(p, F::bfly(p, j, m), F::elem(p, m)))];
      // element 0 of every butterfly has the twiddle exponent 0
      v[m] = F::elem(p, m) == 0 ? x : (INV ? cmulc(x, w[p - 1][m]) : cmul(x, w[p - 1][m]));
    }
    if (p == 1) dft_pass<N, 1, INV>(v);
    if (p == 2) dft_pass<N, (F::P > 2 ? 2 : 1), INV>(v);
  }
}

// Decimation in frequency: v holds layout B on entry, layout A on exit.
template <typename T, int N, bool INV, bool WAVE = false, class Slot>
__device__ __forceinline__ void fft_dif(cplx<T> (&v)[8], cplx<T>* buf0, cplx<T>* buf1, int& parity, const Slot& slot,
                                        int j, const cplx<T> (&w)[RegFFT<N>::P - 1][8]) {
  using F = RegFFT<N>;
  using V = cplx<T>;
#pragma unroll
  for (int p = F::P - 1; p >= 1; --p) {
    if (p == 2) dft_pass<N, (F::P > 2 ? 2 : 1), INV>(v);
    if (p == 1) dft_pass<N, 1, INV>(v);
    V* buf = (parity++ & 1) ? buf1 : buf0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const V y = F::elem(p, m) == 0 ? v[m] : (INV ? cmulc(v[m], w[p - 1][m]) : cmul(v[m], w[p - 1][m]));
      buf[slot(F::rpos(p, F::bfly(p, j, m), F::elem(p, m)))] = y;
    }
    xsync<WAVE>();
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = buf[slot(F::wpos(p - 1, F::bfly(p - 1, j, m), F::elem(p - 1, m)))];
  }
  dft_pass<N, 0, INV>(v);
}

// Row tiles (axis 2, contiguous): lane = T * row + j; pitch N + N/8 with a skew
// of one slot per 8 points.  Column tiles (axes 0 and 1): lane = line + LINES * j.
template <int N> struct RowSlotR {
  int base;
  __device__ __forceinline__ int operator()(int n) const { return base + n + (n >> 3); }
};
template <int N> struct ColSlotR {
  int line;
  __device__ __forceinline__ int operator()(int n) const { return n * RegFFT<N>::LINES + line; }
};

// Staging slot of (i2, line) in a row tile's N x LINES block of the
// transposed work layout: the line index XOR a swizzle of i2, so that both the
// FFT-side pattern (a wavefront holds 64 / (N/8) lines x N/8 points) and the
// coalesced pattern (runs of LINES consecutive lines per i2) hit distinct LDS
// slots for N = 64 (at most 2-way conflicts for 16, 32, 128).
template <int N> __device__ __forceinline__ int tr_slot(int i2, int ln) {
  constexpr int L = RegFFT<N>::LINES;
  return i2 * L + (ln ^ ((((i2 & 7) << 1) | ((i2 & 1) << 4)) & (L - 1)));
}

// ---------------------------------------------------------------------------
// K, first pass (same contract as k_strain_row; tpv = n0 n1 / LINES)
// ---------------------------------------------------------------------------
// TR: write the strain to the transposed work layout [vec][c][i2][i0 i1] (the
// (i0, i1) planes contiguous, for the plane pass) instead of [vec][c][i0 i1][i2];
// the tile is staged through LDS so that every store writes runs of LINES
// consecutive (i0, i1) positions.
template <typename T, int N, int MODE, bool TR = false>
__global__ __launch_bounds__(NT) void k_strain_row_r(const cplx<T>* __restrict__ U, cplx<T>* __restrict__ Pp,
                                                     cplx<T>* __restrict__ W, const double* __restrict__ qtab,
                                                     int n0, int n1, long nvox, int tpv,
                                                     const cplx<T>* __restrict__ tw, const int* __restrict__ active,
                                                     const double* __restrict__ beta, C21v<T> C0, CellSel csel) {
  using V = cplx<T>;
  using F = RegFFT<N>;
  __shared__ V lds[2][F::BUF];
  __shared__ V stage[TR ? N * F::LINES : 1];
  const int v = blockIdx.x / tpv;
  const int tile = blockIdx.x - v * tpv;
  if (active && !active[v]) return;
  const int tid = threadIdx.x;
  const int j = tid % F::T, line = tid / F::T;
  const int row = tile * F::LINES + line;
  const int i0 = row / n1, i1 = row - i0 * n1;
  const double* q = qtab + (size_t)v * (n0 + n1 + N);
  const T qa = (T)q[i0], qb = (T)q[n0 + i1];
  T qc[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) qc[m] = (T)q[n0 + n1 + F::posA(j, m)];
  V w[F::P - 1][8];
  load_twr<T, N>(w, tw, j);
  const size_t rbase = (size_t)row * N;
  V u[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int m = 0; m < 8; ++m) u[c][m] = U[((size_t)v * 3 + c) * nvox + rbase + F::posA(j, m)];
  if (MODE == 1) {
    const T bt = (T)beta[v];
    const C21v<T> C0c = cell_c0<T>(csel, v, C0);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      V in[3] = {u[0][m], u[1][m], u[2][m]}, z[3];
      precond3<T, V>(C0c, qa, qb, qc[m], in, z);
      const size_t o = rbase + F::posA(j, m);
      if (bt != T(0)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) z[c] = caxpy(z[c], bt, Pp[((size_t)v * 3 + c) * nvox + o]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Pp[((size_t)v * 3 + c) * nvox + o] = z[c];
        u[c][m] = z[c];
      }
    }
  }
  const RowSlotR<N> slot{line * (N + N / 8)};
  int parity = 0;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    V e[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      switch (c) {
        case 0: e[m] = cscale(u[0][m], qa); break;
        case 1: e[m] = cscale(u[1][m], qb); break;
        case 2: e[m] = cscale(u[2][m], qc[m]); break;
        case 3: e[m] = cadd(cscale(u[1][m], qc[m]), cscale(u[2][m], qb)); break;
        case 4: e[m] = cadd(cscale(u[0][m], qc[m]), cscale(u[2][m], qa)); break;
        default: e[m] = cadd(cscale(u[0][m], qb), cscale(u[1][m], qa)); break;
      }
    }
    fft_dit<T, N, true>(e, lds[0], lds[1], parity, slot, j, w);
    if (TR) {
      // the previous component's reads of `stage` finished before the
      // workgroup barrier inside this component's transform
      const long n01 = nvox / N;
#pragma unroll
      for (int m = 0; m < 8; ++m) stage[tr_slot<N>(F::posB(j, m), line)] = e[m];
      __syncthreads();
      cplx<T>* Wc = W + ((size_t)v * 6 + c) * nvox + (size_t)tile * F::LINES;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int el = s * NT + tid, i2 = el / F::LINES, ln = el % F::LINES;
        Wc[(size_t)i2 * n01 + ln] = stage[tr_slot<N>(i2, ln)];
      }
    } else {
#pragma unroll
      for (int m = 0; m < 8; ++m) W[((size_t)v * 6 + c) * nvox + rbase + F::posB(j, m)] = e[m];
    }
  }
}

// ---------------------------------------------------------------------------
// K, last pass (same contract as k_row_div; partials per tile)
// ---------------------------------------------------------------------------
// TR: read the stress from the transposed work layout (see k_strain_row_r),
// with coalesced loads staged through LDS.
template <typename T, int N, int MODE, bool TR = false>
__global__ __launch_bounds__(NT) void k_row_div_r(const cplx<T>* __restrict__ W, cplx<T>* __restrict__ Y,
                                                  const double* __restrict__ qtab, int n0, int n1, long nvox,
                                                  int tpv, const cplx<T>* __restrict__ tw,
                                                  const int* __restrict__ active, const cplx<T>* __restrict__ Pp,
                                                  PcgDev pd, T oscale) {
  using V = cplx<T>;
  using F = RegFFT<N>;
  __shared__ V lds[2][F::BUF];
  __shared__ V stage[TR ? N * F::LINES : 1];
  __shared__ double sh[NT / 64];
  const int v = blockIdx.x / tpv;
  const int tile = blockIdx.x - v * tpv;
  if (active && !active[v]) return;
  const int tid = threadIdx.x;
  const int j = tid % F::T, line = tid / F::T;
  const int row = tile * F::LINES + line;
  const int i0 = row / n1, i1 = row - i0 * n1;
  const double* q = qtab + (size_t)v * (n0 + n1 + N);
  const T qa = (T)q[i0], qb = (T)q[n0 + i1];
  T qc[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) qc[m] = (T)q[n0 + n1 + F::posB(j, m)];
  V w[F::P - 1][8];
  load_twr<T, N>(w, tw, j);
  const size_t rbase = (size_t)row * N;
  const RowSlotR<N> slot{line * (N + N / 8)};
  int parity = 0;
  V acc[3][8];
#pragma unroll
  for (int m = 0; m < 8; ++m) acc[0][m] = acc[1][m] = acc[2][m] = V{0, 0};
  const long n01 = nvox / N;
  // TR: element s of this thread is (i2, line) = divmod(s NT + tid, LINES) of the tile
  auto widx = [&](int c, int m) -> size_t {
    if (TR) {
      const int el = m * NT + tid;
      return ((size_t)v * 6 + c) * nvox + (size_t)(el / F::LINES) * n01 + (size_t)tile * F::LINES + el % F::LINES;
    }
    return ((size_t)v * 6 + c) * nvox + rbase + F::posA(j, m);
  };
  V nxt[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) nxt[m] = W[widx(0, m)];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    V e[8];
    if (TR) {
      // the previous component's reads of `stage` finished before the
      // workgroup barrier inside its transform
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int el = m * NT + tid;
        stage[tr_slot<N>(el / F::LINES, el % F::LINES)] = nxt[m];
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < 8; ++m) e[m] = stage[tr_slot<N>(F::posA(j, m), line)];
    } else {
#pragma unroll
      for (int m = 0; m < 8; ++m) e[m] = nxt[m];
    }
    if (c < 5) {
#pragma unroll
      for (int m = 0; m < 8; ++m) nxt[m] = W[widx(c + 1, m)];
    }
    fft_dit<T, N, false>(e, lds[0], lds[1], parity, slot, j, w);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      switch (c) {
        case 0: acc[0][m] = caxpy(acc[0][m], qa, e[m]); break;
        case 1: acc[1][m] = caxpy(acc[1][m], qb, e[m]); break;
        case 2: acc[2][m] = caxpy(acc[2][m], qc[m], e[m]); break;
        case 3: acc[1][m] = caxpy(acc[1][m], qc[m], e[m]); acc[2][m] = caxpy(acc[2][m], qb, e[m]); break;
        case 4: acc[0][m] = caxpy(acc[0][m], qc[m], e[m]); acc[2][m] = caxpy(acc[2][m], qa, e[m]); break;
        default: acc[0][m] = caxpy(acc[0][m], qb, e[m]); acc[1][m] = caxpy(acc[1][m], qa, e[m]); break;
      }
    }
  }
  double part = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const size_t o = ((size_t)v * 3 + c) * nvox + rbase + F::posB(j, m);
      const V ov = cscale(acc[c][m], oscale);
      Y[o] = ov;
      if (MODE == 1) {
        const V pv = Pp[o];
        part += (double)pv.x * (double)ov.x + (double)pv.y * (double)ov.y;
      }
    }
  if (MODE == 1) {
    const double vals[1] = {part};
    store_partials<1>(vals, pd.partial, v, tile, pd.max_blocks, sh);
  }
}

// ---------------------------------------------------------------------------
// FFT along axis 1 (stride n2, n2 % LINES == 0), in place; lines are (plane,
// column) with plane = (component, i0).  tpv = planes * n2 / LINES.
// ---------------------------------------------------------------------------
template <typename T, int N, bool INV, int PCG = 0>
__global__ __launch_bounds__(NT) void k_axis1_r(cplx<T>* __restrict__ X, int n2, long vec_stride, int tpv,
                                                const cplx<T>* __restrict__ tw, const int* __restrict__ active) {
  using V = cplx<T>;
  using F = RegFFT<N>;
  __shared__ V lds[F::NBUF][F::BUFC];
  const int v = blockIdx.x / tpv;
  if (active && !active[v]) return;
  const int tile = blockIdx.x - v * tpv;
  const int tid = threadIdx.x;
  const int line = tid % F::LINES, j = tid / F::LINES;
  const int tpp = n2 / F::LINES;
  const int plane = tile / tpp;
  const int col = (tile - plane * tpp) * F::LINES + line;
  V* base = X + (size_t)v * vec_stride + (size_t)plane * N * n2 + col;
  V w[F::P - 1][8];
  load_twr<T, N>(w, tw, j);
  V e[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) e[m] = base[(size_t)F::posA(j, m) * n2];
  int parity = 0;
  fft_dit<T, N, INV>(e, lds[0], lds[F::NBUF - 1], parity, ColSlotR<N>{line}, j, w);
#pragma unroll
  for (int m = 0; m < 8; ++m) base[(size_t)F::posB(j, m) * n2] = e[m];
}

// ---------------------------------------------------------------------------
// Axis 0 (same contract as k_axis0_op; n12 % LINES == 0, NC nvox < 2^31):
// inverse FFT (layout A -> B), stiffness contraction (OP 0) or density
// scaling (OP 1) at the layout-B points, forward FFT back to layout A.
// ---------------------------------------------------------------------------
// FP32: at most 168 VGPRs, so that 3 wavefronts fit per SIMD (the 6 x 8 points
// take 96; the loads and stores hold no 64-bit addresses).
template <typename T, int N, int OP, int PCG = 0>
__global__ __launch_bounds__(NT, sizeof(T) == 4 ? 3 : 2) void k_axis0_op_r(cplx<T>* __restrict__ X, long n12, long nvox, int tpv,
                                                      const uint16_t* __restrict__ gmap, const T* __restrict__ Ctab,
                                                      T scale, const cplx<T>* __restrict__ tw,
                                                      const int* __restrict__ active, CellSel csel) {
  using V = cplx<T>;
  using F = RegFFT<N>;
  constexpr int NC = OP == 0 ? 6 : 3;
  __shared__ V lds[2][F::BUFC];
  const int v = blockIdx.x / tpv;
  if (active && !active[v]) return;
  const int tile = blockIdx.x - v * tpv;
  const int tid = threadIdx.x;
  const int line = tid % F::LINES, j = tid / F::LINES;
  const int pos = tile * F::LINES + line;
  V w[F::P - 1][8];
  load_twr<T, N>(w, tw, j);
  // 32-bit offsets within the vector (NC * nvox < 2^31, checked by the host):
  // point (c, m) of this thread sits at lo + c cs + m T s12, a per-thread base
  // plus a uniform offset, so no 64-bit address is held per load
  cplx<T>* Xv = X + (size_t)v * NC * nvox;
  const uint16_t* __restrict__ gmv = gmap + csel.goff(v);   // this vector's cell
  const int s12 = (int)n12;
  const uint32_t cs = (uint32_t)nvox, ms = (uint32_t)(F::T * n12);
  uint32_t lo = (uint32_t)pos + (uint32_t)j * (uint32_t)n12;
  V x[NC][8];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int m = 0; m < 8; ++m) x[c][m] = Xv[lo + c * cs + m * ms];
  const ColSlotR<N> slot{line};
  int parity = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) fft_dit<T, N, true>(x[c], lds[0], lds[1], parity, slot, j, w);
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int g = gmv[pos + F::posB(j, m) * s12];
    if (OP == 0) {
      T cg[21];
#pragma unroll
      for (int i = 0; i < 21; ++i) cg[i] = Ctab[g * 21 + i];
      V e[6], sg[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = x[c][m];
      contract6<T, V>(cg, e, sg, scale);
#pragma unroll
      for (int c = 0; c < 6; ++c) x[c][m] = sg[c];
    } else {
      const T rs = Ctab[g] * scale;
#pragma unroll
      for (int c = 0; c < NC; ++c) x[c][m] = cscale(x[c][m], rs);
    }
    // keep the table loads of one point at a time in flight (register pressure)
    asm volatile("" ::: "memory");
  }
  // the base again, opaque: the store addresses are formed anew, not kept in
  // registers since the loads
  asm volatile("" : "+v"(lo));
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    fft_dif<T, N, false>(x[c], lds[0], lds[1], parity, slot, j, w);
#pragma unroll
    for (int m = 0; m < 8; ++m) Xv[lo + c * cs + m * ms] = x[c][m];
  }
}

// Two length-64 transforms at once with wavefront-local exchanges (one buffer
// each): the butterflies of one overlap the LDS latency of the other.  The
// fence before the writes keeps them behind the reads of the previous exchange
// in the same buffers.
// twf(m): twiddle of register m in pass 1.
template <typename T, bool INV, class Slot, class TwF>
__device__ __forceinline__ void fft64_pair(cplx<T> (&a)[8], cplx<T> (&b)[8], cplx<T>* bufa, cplx<T>* bufb,
                                           const Slot& slot, int j, const TwF& twf) {
  using F = RegFFT<64>;
  using V = cplx<T>;
  dft_pass<64, 0, INV>(a);
  dft_pass<64, 0, INV>(b);
  xsync<true>();
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int o = slot(F::wpos(0, F::bfly(0, j, m), F::elem(0, m)));
    bufa[o] = a[m];
    bufb[o] = b[m];
  }
  xsync<true>();
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int o = slot(F::rpos(1, F::bfly(1, j, m), F::elem(1, m)));
    const V xa = bufa[o], xb = bufb[o];
    if (F::elem(1, m) == 0) {
      a[m] = xa;
      b[m] = xb;
    } else {
      const V t = twf(m);
      a[m] = INV ? cmulc(xa, t) : cmul(xa, t);
      b[m] = INV ? cmulc(xb, t) : cmul(xb, t);
    }
  }
  dft_pass<64, 1, INV>(a);
  dft_pass<64, 1, INV>(b);
}
template <typename T, bool INV, class Slot>
__device__ __forceinline__ void fft64_dit_pair(cplx<T> (&a)[8], cplx<T> (&b)[8], cplx<T>* bufa, cplx<T>* bufb,
                                               const Slot& slot, int j, const cplx<T> (&w)[1][8]) {
  fft64_pair<T, INV>(a, b, bufa, bufb, slot, j, [&](int m) { return w[0][m]; });
}

// ---------------------------------------------------------------------------
// Plane pass for n0 = n1 = 64 on the transposed work layout: a workgroup takes
// the 64 x 64 (i0, i1) planes of all six strain components, one (vector, i2)
// plane after another: inverse 2D FFT (axis 1 then axis 0, register transforms
// with a transposition through LDS between them), stiffness contraction,
// forward 2D FFT, and the stress written back in place: the three middle
// passes of K in one read and one write of the work array.
//
// One workgroup per CU holds a plane in registers (two planes would not fit the
// register file).  The workgroups are persistent: they take the planes of the
// active vectors (all vectors when `active` is null) in turn, ordinal a =
// blockIdx.x, blockIdx.x + gridDim.x, ..., and as soon as a component pair of a
// plane is stored, the same registers receive that pair of the next plane, so the
// loads of the next plane overlap the transforms of this one.  The active vectors
// are first listed in LDS, so that the planes are dealt out evenly whichever
// vectors have converged (beyond PLANE_LIST vectors the ordinal runs over all
// planes and those of inactive vectors are skipped).
// ---------------------------------------------------------------------------
constexpr int PLANE_NT = 512;       // 64 lines x 8 threads
// Transposition slot of (i0, i1): row i0, column i1 XOR a swizzle of i0's low
// bits.  Lanes of a wave cover 8 lines x 8 points (write: i0 = line; read:
// i0 = point), and the swizzle spreads both patterns over distinct 8-byte slots
// modulo 16 within each 16 lanes and modulo 32 within each 32 lanes.
__device__ __forceinline__ int plane_tslot(int i0, int i1) {
  const int f = ((i0 & 2) | (i0 & 4) | ((i0 & 1) << 3) | ((i0 & 2) << 3));
  return i0 * 64 + (i1 ^ f);
}
// The two axes have the same length, so one twiddle set serves both.
// CL: the stiffness table (G <= PLANE_CL_MAX grains) is staged in LDS; the
// grain indices of a plane are loaded when its transforms start, so neither
// load is waited for in the contraction.
constexpr int PLANE_CL_MAX = 256;
constexpr int PLANE_LIST = 256;     // vectors listed in LDS
template <typename T, int PCG = 0, bool CL = false>
__global__ __launch_bounds__(PLANE_NT, 1) void k_plane64(cplx<T>* __restrict__ W, int n2, int nplanes, long nvox,
                                                         const uint16_t* __restrict__ gmapT, const T* __restrict__ Ctab,
                                                         int ngrains, T scale, const cplx<T>* __restrict__ tw,
                                                         const int* __restrict__ active, CellSel csel) {
  using V = cplx<T>;
  constexpr int NB = 64 * (64 + 8);   // 64 lines at the skewed row pitch (FFT exchanges, wavefront-local)
  __shared__ V lds[2][NB];
  __shared__ V tr[2][64 * 64];        // transpositions of a pair of components (workgroup-wide)
  __shared__ T cl[CL ? PLANE_CL_MAX * 21 : 1];
  __shared__ int alist[PLANE_LIST];
  __shared__ int nact_s;
  const int tid = threadIdx.x;
  const int nvec = nplanes / n2;
  const bool listed = active != nullptr && nvec <= PLANE_LIST;
  if (listed) {
    if (tid < 64) {   // wavefront 0: the active vectors in order
      int base = 0;
      for (int c = 0; c < nvec; c += 64) {
        const int v = c + tid;
        const bool f = v < nvec && active[v] != 0;
        const unsigned long long m = __ballot(f);
        if (f) alist[base + __popcll(m & ((1ull << tid) - 1ull))] = v;
        base += __popcll(m);
      }
      if (tid == 0) nact_s = base;
    }
    __syncthreads();
  }
  const int nlisted = listed ? nact_s * n2 : 0;
  // plane of ordinal a (uniform), or nplanes when there is none; unlisted, a is
  // advanced past the planes of inactive vectors
  const auto plane_at = [&](int& a) {
    if (listed) {
      if (a >= nlisted) return nplanes;
      const int i = a / n2;
      return alist[i] * n2 + (a - i * n2);
    }
    while (a < nplanes && active && !active[a / n2]) a += gridDim.x;
    return a < nplanes ? a : nplanes;
  };
  int a = blockIdx.x;
  int p = plane_at(a);
  if (p >= nplanes) return;
  if (CL)   // with the scale folded in; visible after the first barrier
    for (int i = tid; i < ngrains * 21; i += PLANE_NT) cl[i] = Ctab[i] * scale;
  const T* __restrict__ Cg = CL ? cl : Ctab;
  V w[1][8];
  load_twr<T, 64>(w, tw, tid & 7);
  const auto plane_ptr = [&](int q) {
    const int v = q / n2;
    return W + (size_t)v * 6 * nvox + (size_t)(q - v * n2) * 4096;
  };
  V x[6][8];
  {
    const int line = tid >> 3, j = tid & 7;
    const V* Wv = plane_ptr(p);
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int m = 0; m < 8; ++m) x[c][m] = Wv[(size_t)c * nvox + line * 64 + j + 8 * m];  // (i0 = line, i1 = j + 8m)
  }
  for (;;) {
    // the lane's position, opaque to the compiler: every address below is
    // recomputed per plane instead of being hoisted out of the loop, which would
    // hold some hundred registers for the whole loop
    int line = tid >> 3, j = tid & 7;
    asm volatile("" : "+v"(line), "+v"(j));
    const RowSlotR<64> slot{line * (64 + 8)};
    int an = a + gridDim.x;
    const int pn = plane_at(an);
    const int i2 = p % n2;
    V* Wv = plane_ptr(p);
    int gm[8];                    // grain of point (i0 = j + 8m, i1 = line)
    const uint16_t* __restrict__ gmp = gmapT + csel.goff(p / n2) + (size_t)i2 * 4096;   // this plane's cell
#pragma unroll
    for (int m = 0; m < 8; ++m) gm[m] = gmp[(j + 8 * m) * 64 + line];
#pragma unroll
    for (int c = 0; c < 6; c += 2) {
      fft64_dit_pair<T, true>(x[c], x[c + 1], lds[0], lds[1], slot, j, w);   // along i1
      __syncthreads();            // every wavefront has read the previous transposition
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        tr[0][plane_tslot(line, j + 8 * m)] = x[c][m];
        tr[1][plane_tslot(line, j + 8 * m)] = x[c + 1][m];
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < 8; ++m) {                    // (i0 = j + 8m, i1 = line)
        x[c][m] = tr[0][plane_tslot(j + 8 * m, line)];
        x[c + 1][m] = tr[1][plane_tslot(j + 8 * m, line)];
      }
      fft64_dit_pair<T, true>(x[c], x[c + 1], lds[0], lds[1], slot, j, w);   // along i0
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      T cg[21];
#pragma unroll
      for (int i = 0; i < 21; ++i) cg[i] = Cg[gm[m] * 21 + i];
      V e[6], sg[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = x[c][m];
      contract6<T, V>(cg, e, sg, CL ? T(1) : scale);
#pragma unroll
      for (int c = 0; c < 6; ++c) x[c][m] = sg[c];
      // one point's stiffness at a time: the scheduler would otherwise issue the
      // loads of all eight points at once and spill them
      __builtin_amdgcn_sched_barrier(0);
    }
    // inverse 2D FFT and store, pair by pair; PF: each pair followed by the loads
    // of that pair of the next plane into the same registers (two instances, so
    // that the stored and the loaded values are never live at once)
    const auto finish = [&](auto PF, const V* Wn) {
#pragma unroll
      for (int c = 0; c < 6; c += 2) {
        fft64_dit_pair<T, false>(x[c], x[c + 1], lds[0], lds[1], slot, j, w);   // along i0
        __syncthreads();          // every wavefront has read the previous transposition
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          tr[0][plane_tslot(j + 8 * m, line)] = x[c][m];
          tr[1][plane_tslot(j + 8 * m, line)] = x[c + 1][m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m) {                  // (i0 = line, i1 = j + 8m)
          x[c][m] = tr[0][plane_tslot(line, j + 8 * m)];
          x[c + 1][m] = tr[1][plane_tslot(line, j + 8 * m)];
        }
        fft64_dit_pair<T, false>(x[c], x[c + 1], lds[0], lds[1], slot, j, w);   // along i1
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          Wv[(size_t)c * nvox + line * 64 + j + 8 * m] = x[c][m];
          Wv[(size_t)(c + 1) * nvox + line * 64 + j + 8 * m] = x[c + 1][m];
        }
        if (decltype(PF)::value) {
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            x[c][m] = Wn[(size_t)c * nvox + line * 64 + j + 8 * m];
            x[c + 1][m] = Wn[(size_t)(c + 1) * nvox + line * 64 + j + 8 * m];
          }
        }
      }
    };
    if (pn >= nplanes) {
      finish(std::false_type{}, Wv);
      break;
    }
    finish(std::true_type{}, plane_ptr(pn));
    p = pn;
    a = an;
  }
}

// which lengths / tilings take the register kernels
inline bool reg_len(int n) { return n == 16 || n == 32 || n == 64 || n == 128 || n == 256; }
inline int reg_lines(int n) { return NT / (n / 8); }

}  // namespace bw
