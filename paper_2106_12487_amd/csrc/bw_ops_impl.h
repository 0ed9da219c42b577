// Operator kernels of the Bloch method, templated on the working precision T.
//
// Data layout: a batch of vectors is [nvec][3][n0][n1][n2] complex (n2 fastest);
// the strain / stress work array is [nvec][6][n0][n1][n2].  The 3D transforms
// are split into one kernel per axis; the pointwise steps are fused into them:
//
//   K(k) u (Sec. 3.2 eq. hatA, six independent strain components by the minor
//   symmetry of C):
//     k_strain_row   e^ = B(q) u^ (Voigt strain), inverse FFT along axis 2
//     k_axis1        inverse FFT along axis 1
//     k_axis0_op     inverse FFT along axis 0, s = C(x) e, forward FFT axis 0
//     k_axis1        forward FFT along axis 1
//     k_row_div      forward FFT along axis 2, out = B(q)^T s^ (divergence)
//   M u (eq. hatM): the same chain with three components and s = rho(x) u.
//
// One component of a tile is staged in LDS at a time; every component of the
// points a thread owns stays in its registers, so a pass reads and writes each
// word of its input and output once.  The 1/(n0 n1 n2) of the inverse
// transform and the caller's scale are folded into the pointwise step.
#pragma once
#include <type_traits>

#include "bw_internal.h"

namespace bw {

template <typename T> struct C21v { T c[21]; };

// index of a precision's FFT schedule in a cell (0: FP32 kernels, 1: FP64)
template <typename T> constexpr int tsel = sizeof(T) == 8 ? 1 : 0;

// the reference stiffness C0 of vector v's cell (the kernel's own C0 for one cell)
template <typename T> __device__ __forceinline__ C21v<T> cell_c0(const CellSel& cs, int v, const C21v<T>& C0) {
  const T* tab;
  if constexpr (sizeof(T) == 4) tab = (const T*)cs.c0tab32;
  else tab = (const T*)cs.c0tab64;
  if (cs.n <= 1 || !tab) return C0;
  C21v<T> c;
  const T* row = tab + (size_t)cs.cell(v) * 21;
#pragma unroll
  for (int i = 0; i < 21; ++i) c.c[i] = row[i];
  return c;
}

// Voigt upper-triangle index of (a, b)
__host__ __device__ constexpr int vidx(int a, int b) {
  return a <= b ? a * 6 - (a * (a - 1)) / 2 + (b - a) : b * 6 - (b * (b - 1)) / 2 + (a - b);
}

// sigma = C e for one voxel (C symmetric 6x6 given by its 21 upper entries)
template <typename T, typename V>
__device__ __forceinline__ void contract6(const T* __restrict__ c, const V* e, V* s, T scale) {
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    T sx = 0, sy = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const T cab = c[vidx(a, b)];
      sx += cab * e[b].x;
      sy += cab * e[b].y;
    }
    s[a] = V{sx * scale, sy * scale};
  }
}

// z = P(C0, q)^-1 r with P_ik = C0_ijkl q_j q_l (Sec. 3.3 eqs. matrixP, precond);
// z = 0 where q = 0.
template <typename T, typename V>
__device__ __forceinline__ void precond3(const C21v<T>& C0, T q0, T q1, T q2, const V* r, V* z) {
  if (q0 == T(0) && q1 == T(0) && q2 == T(0)) {
    z[0] = z[1] = z[2] = V{0, 0};
    return;
  }
  // B(q): rows = Voigt strain components, columns = displacement components
  const T B[6][3] = {{q0, 0, 0}, {0, q1, 0}, {0, 0, q2}, {0, q2, q1}, {q2, 0, q0}, {q1, q0, 0}};
  T CB[6][3];
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T acc = 0;
#pragma unroll
      for (int b = 0; b < 6; ++b) acc += C0.c[vidx(a, b)] * B[b][k];
      CB[a][k] = acc;
    }
  T P[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T acc = 0;
#pragma unroll
      for (int a = 0; a < 6; ++a) acc += B[a][i] * CB[a][k];
      P[i][k] = acc;
    }
  const T a = P[0][0], b = P[0][1], c = P[0][2], d = P[1][1], e = P[1][2], f = P[2][2];
  const T A00 = d * f - e * e, A01 = c * e - b * f, A02 = b * e - c * d;
  const T A11 = a * f - c * c, A12 = b * c - a * e, A22 = a * d - b * b;
  const T inv = T(1) / (a * A00 + b * A01 + c * A02);
  const T Ai[3][3] = {{A00, A01, A02}, {A01, A11, A12}, {A02, A12, A22}};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T zx = 0, zy = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      zx += Ai[i][k] * r[k].x;
      zy += Ai[i][k] * r[k].y;
    }
    z[i] = V{zx * inv, zy * inv};
  }
}

// ---------------------------------------------------------------------------
// reductions: wave64 shuffles, LDS across waves, deterministic last-block sum
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum (valid in thread 0).  `sh` needs NT/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) s += sh[i];
  return s;
}

__device__ __forceinline__ double coherent_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Writes this block's NV partial sums for vector v (plain stores).  A finalize
// kernel launched afterwards sums them in block order, so the result does not
// depend on scheduling and no device-wide fence is needed inside the kernel.
template <int NV>
__device__ __forceinline__ void store_partials(const double (&vals)[NV], double* partial, int v, int blk, int maxb,
                                               double* sh) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double s = block_sum(vals[i], sh);
    if (threadIdx.x == 0) partial[((size_t)v * maxb + blk) * NV + i] = s;
  }
}

// Sum of the NV partials of vector v over nblk blocks in block order (valid in
// thread 0 of a one-block-per-vector finalize kernel).
template <int NV>
__device__ __forceinline__ void sum_partials(double (&tot)[NV], const double* partial, int v, int nblk, int maxb,
                                             double* sh) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double acc = 0;
    for (int b = threadIdx.x; b < nblk; b += NT) acc += partial[((size_t)v * maxb + b) * NV + i];
    tot[i] = block_sum(acc, sh);
  }
}

// finalize ops
enum FinOp { FIN_ALPHA = 0, FIN_BETA = 1, FIN_RESID = 2, FIN_RESTART = 3 };

static __global__ __launch_bounds__(NT) void k_finalize(int op, int nblk, PcgDev pd, const int* __restrict__ mask,
                                                 double* rr_out, double* bb_out) {
  __shared__ double sh[NT / 64];
  const int v = blockIdx.x;
  if (op == FIN_ALPHA) {
    if (!pd.active[v]) return;
    double tot[1];
    sum_partials<1>(tot, pd.partial, v, nblk, pd.max_blocks, sh);
    if (threadIdx.x == 0) {
      pd.pAp[v] = tot[0];
      pd.alpha[v] = tot[0] > 0 ? pd.rz[v] / tot[0] : 0.0;
    }
  } else if (op == FIN_BETA) {
    if (!pd.active[v]) return;
    double tot[2];
    sum_partials<2>(tot, pd.partial, v, nblk, pd.max_blocks, sh);
    if (threadIdx.x == 0) {
      const double old = pd.rz[v];
      pd.beta[v] = old != 0.0 ? tot[0] / old : 0.0;
      pd.rz[v] = tot[0];
      pd.rr[v] = tot[1];
      const int it = pd.iters[v] + 1;
      pd.iters[v] = it;
      if (tot[1] <= pd.bb[v] || it >= pd.maxit) pd.active[v] = 0;
    }
  } else if (op == FIN_RESID) {
    double tot[2];
    sum_partials<2>(tot, pd.partial, v, nblk, pd.max_blocks, sh);
    if (threadIdx.x == 0) {
      rr_out[v] = tot[0];
      if (bb_out) bb_out[v] = tot[1];
    }
  } else {
    if (!mask[v]) return;
    double tot[1];
    sum_partials<1>(tot, pd.partial, v, nblk, pd.max_blocks, sh);
    if (threadIdx.x == 0) {
      pd.rz[v] = tot[0];
      pd.beta[v] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// tile bookkeeping for row kernels (axis 2, contiguous)
// ---------------------------------------------------------------------------
struct RowTile {
  int NR, lsh, tpv;  // rows per tile, log2(NR), tiles per vector
};
struct ColTile {
  int LT, lsh, tpv;  // lines per tile, log2(LT), tiles per vector
};

// ---------------------------------------------------------------------------
// K, first pass: strain (optionally preceded by the PCG direction update
// p = P^ r + beta p) and inverse FFT along axis 2.
// MODE 0: u = U.  MODE 1: U = r, P = p (updated in place), u = p_new.
// ---------------------------------------------------------------------------
template <typename T, int N2, int MODE>
__global__ __launch_bounds__(NT) void k_strain_row(const cplx<T>* __restrict__ U, cplx<T>* __restrict__ Pp,
                                                   cplx<T>* __restrict__ W, const double* __restrict__ qtab,
                                                   int n0, int n1, long nvox, RowTile rt,
                                                   const cplx<T>* __restrict__ tw, const int* __restrict__ active,
                                                   const double* __restrict__ beta, C21v<T> C0, CellSel csel) {
  using V = cplx<T>;
  constexpr int TP = TileCfg<T>::TP;
  constexpr int PPT = TP / NT;
  __shared__ V lds[TP + N2];
  const int v = blockIdx.x / rt.tpv;
  const int tile = blockIdx.x - v * rt.tpv;
  if (active && !active[v]) return;
  const int tid = threadIdx.x;
  const int npts = rt.NR * N2;
  const int P = rt.NR + 1;
  const double* q = qtab + (size_t)v * (n0 + n1 + N2);
  T bt = 0;
  if (MODE == 1) bt = (T)beta[v];
  const C21v<T> C0c = MODE == 1 ? cell_c0<T>(csel, v, C0) : C0;
  V u[3][PPT];
  T qa[PPT], qb[PPT], qc[PPT];
  int off[PPT];
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int idx = tid + s * NT;
    off[s] = -1;
    if (idx < npts) {
      const int rl = idx / N2, n = idx - rl * N2;
      const int row = tile * rt.NR + rl;
      const int i0 = row / n1, i1 = row - i0 * n1;
      off[s] = row * N2 + n;
      qa[s] = (T)q[i0];
      qb[s] = (T)q[n0 + i1];
      qc[s] = (T)q[n0 + n1 + n];
      V w[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c] = U[((size_t)v * 3 + c) * nvox + off[s]];
      if (MODE == 1) {
        V z[3];
        precond3<T, V>(C0c, qa[s], qb[s], qc[s], w, z);
        if (bt != T(0)) {
#pragma unroll
          for (int c = 0; c < 3; ++c) z[c] = caxpy(z[c], bt, Pp[((size_t)v * 3 + c) * nvox + off[s]]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Pp[((size_t)v * 3 + c) * nvox + off[s]] = z[c];
          w[c] = z[c];
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) u[c][s] = w[c];
    }
  }
#pragma unroll 1
  for (int c = 0; c < 6; ++c) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      if (off[s] >= 0) {
        const int idx = tid + s * NT;
        const int rl = idx / N2, n = idx - rl * N2;
        V e;
        switch (c) {
          case 0: e = cscale(u[0][s], qa[s]); break;
          case 1: e = cscale(u[1][s], qb[s]); break;
          case 2: e = cscale(u[2][s], qc[s]); break;
          case 3: e = cadd(cscale(u[1][s], qc[s]), cscale(u[2][s], qb[s])); break;
          case 4: e = cadd(cscale(u[0][s], qc[s]), cscale(u[2][s], qa[s])); break;
          default: e = cadd(cscale(u[0][s], qb[s]), cscale(u[1][s], qa[s])); break;
        }
        lds[n * P + rl] = e;
      }
    }
    __syncthreads();
    lds_fft<T, N2, true, NT, TP>(lds, P, rt.NR, rt.lsh, tw, tid);
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      if (off[s] >= 0) {
        const int idx = tid + s * NT;
        const int rl = idx / N2, n = idx - rl * N2;
        W[((size_t)v * 6 + c) * nvox + off[s]] = lds[n * P + rl];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Last pass of K: forward FFT along axis 2 and divergence out_i = q_j s^_ij.
// MODE 1 also forms <p, K p> (FP64) and, in the last block of the vector,
// alpha = <r, z> / <p, K p>.
// ---------------------------------------------------------------------------
template <typename T, int N2, int MODE>
__global__ __launch_bounds__(NT) void k_row_div(const cplx<T>* __restrict__ W, cplx<T>* __restrict__ Y,
                                                const double* __restrict__ qtab, int n0, int n1, long nvox,
                                                RowTile rt, const cplx<T>* __restrict__ tw,
                                                const int* __restrict__ active, const cplx<T>* __restrict__ Pp,
                                                PcgDev pd, T oscale) {
  using V = cplx<T>;
  constexpr int TP = TileCfg<T>::TP;
  constexpr int PPT = TP / NT;
  __shared__ V lds[TP + N2];
  __shared__ double sh[NT / 64];
  const int v = blockIdx.x / rt.tpv;
  const int tile = blockIdx.x - v * rt.tpv;
  if (active && !active[v]) return;
  const int tid = threadIdx.x;
  const int npts = rt.NR * N2;
  const int P = rt.NR + 1;
  const double* q = qtab + (size_t)v * (n0 + n1 + N2);
  V acc[3][PPT];
  T qa[PPT], qb[PPT], qc[PPT];
  int off[PPT];
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int idx = tid + s * NT;
    off[s] = -1;
    acc[0][s] = acc[1][s] = acc[2][s] = V{0, 0};
    if (idx < npts) {
      const int rl = idx / N2, n = idx - rl * N2;
      const int row = tile * rt.NR + rl;
      const int i0 = row / n1, i1 = row - i0 * n1;
      off[s] = row * N2 + n;
      qa[s] = (T)q[i0];
      qb[s] = (T)q[n0 + i1];
      qc[s] = (T)q[n0 + n1 + n];
    }
  }
#pragma unroll 1
  for (int c = 0; c < 6; ++c) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      if (off[s] >= 0) {
        const int idx = tid + s * NT;
        const int rl = idx / N2, n = idx - rl * N2;
        lds[n * P + rl] = W[((size_t)v * 6 + c) * nvox + off[s]];
      }
    }
    __syncthreads();
    lds_fft<T, N2, false, NT, TP>(lds, P, rt.NR, rt.lsh, tw, tid);
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      if (off[s] >= 0) {
        const int idx = tid + s * NT;
        const int rl = idx / N2, n = idx - rl * N2;
        const V sg = lds[n * P + rl];
        switch (c) {
          case 0: acc[0][s] = caxpy(acc[0][s], qa[s], sg); break;                      // s11
          case 1: acc[1][s] = caxpy(acc[1][s], qb[s], sg); break;                      // s22
          case 2: acc[2][s] = caxpy(acc[2][s], qc[s], sg); break;                      // s33
          case 3: acc[1][s] = caxpy(acc[1][s], qc[s], sg); acc[2][s] = caxpy(acc[2][s], qb[s], sg); break;  // s23
          case 4: acc[0][s] = caxpy(acc[0][s], qc[s], sg); acc[2][s] = caxpy(acc[2][s], qa[s], sg); break;  // s13
          default: acc[0][s] = caxpy(acc[0][s], qb[s], sg); acc[1][s] = caxpy(acc[1][s], qa[s], sg); break; // s12
        }
      }
    }
    __syncthreads();
  }
  double part = 0;
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    if (off[s] >= 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const V o = cscale(acc[c][s], oscale);
        Y[((size_t)v * 3 + c) * nvox + off[s]] = o;
        if (MODE == 1) {
          const V pv = Pp[((size_t)v * 3 + c) * nvox + off[s]];
          part += (double)pv.x * (double)o.x + (double)pv.y * (double)o.y;
        }
      }
    }
  }
  if (MODE == 1) {
    const double vals[1] = {part};
    store_partials<1>(vals, pd.partial, v, tile, pd.max_blocks, sh);
  }
}

// ---------------------------------------------------------------------------
// plain row FFT (axis 2) of NC-component fields: rows are flattened over
// (vector, component, i0, i1); a tile never crosses a component.
// ---------------------------------------------------------------------------
template <typename T, int N2, bool INV>
__global__ __launch_bounds__(NT) void k_row_plain(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst,
                                                  RowTile rt, int rows_per_vec, const cplx<T>* __restrict__ tw,
                                                  const int* __restrict__ active) {
  using V = cplx<T>;
  constexpr int TP = TileCfg<T>::TP;
  constexpr int PPT = TP / NT;
  __shared__ V lds[TP + N2];
  const int v = blockIdx.x / rt.tpv;
  if (active && !active[v]) return;
  const size_t base = ((size_t)v * rows_per_vec + (size_t)(blockIdx.x - v * rt.tpv) * rt.NR) * N2;
  const int tid = threadIdx.x;
  const int npts = rt.NR * N2;
  const int P = rt.NR + 1;
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int idx = tid + s * NT;
    if (idx < npts) {
      const int rl = idx / N2, n = idx - rl * N2;
      lds[n * P + rl] = src[base + idx];
    }
  }
  __syncthreads();
  lds_fft<T, N2, INV, NT, TP>(lds, P, rt.NR, rt.lsh, tw, tid);
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int idx = tid + s * NT;
    if (idx < npts) {
      const int rl = idx / N2, n = idx - rl * N2;
      dst[base + idx] = lds[n * P + rl];
    }
  }
}

// ---------------------------------------------------------------------------
// FFT along axis 1 (stride n2), in place, for NC-component fields.  Lines are
// (plane, column) with plane = (component, i0); a tile holds LT consecutive
// lines (within one plane, or whole consecutive planes).
// ---------------------------------------------------------------------------
template <typename T, int N1, bool INV, int PCG = 0>
__global__ __launch_bounds__(NT) void k_axis1(cplx<T>* __restrict__ X, int n2, long vec_stride, ColTile ct,
                                              const cplx<T>* __restrict__ tw, const int* __restrict__ active) {
  using V = cplx<T>;
  constexpr int TP = TileCfg<T>::TP;
  constexpr int PPT = TP / NT;
  __shared__ V lds[TP];
  const int v = blockIdx.x / ct.tpv;
  if (active && !active[v]) return;
  const int tile = blockIdx.x - v * ct.tpv;
  const int tid = threadIdx.x;
  const int line = tid & (ct.LT - 1);
  const int gl = tile * ct.LT + line;
  const int plane = gl / n2, col = gl - plane * n2;
  cplx<T>* base = X + (size_t)v * vec_stride + (size_t)plane * N1 * n2 + col;
  const int npts = ct.LT * N1;
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int idx = tid + s * NT;
    if (idx < npts) {
      const int n = idx >> ct.lsh;
      lds[n * ct.LT + line] = base[(size_t)n * n2];
    }
  }
  __syncthreads();
  lds_fft<T, N1, INV, NT, TP>(lds, ct.LT, ct.LT, ct.lsh, tw, tid);
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int idx = tid + s * NT;
    if (idx < npts) {
      const int n = idx >> ct.lsh;
      base[(size_t)n * n2] = lds[n * ct.LT + line];
    }
  }
}

// ---------------------------------------------------------------------------
// Axis 0: inverse FFT, pointwise real-space step, forward FFT, in place.
// OP 0: stiffness contraction on 6 Voigt components (Ctab: G x 21).
// OP 1: density scaling on 3 components (Ctab: G densities).
// ---------------------------------------------------------------------------
template <typename T, int N0, int OP, int PCG = 0>
__global__ __launch_bounds__(NT) void k_axis0_op(cplx<T>* __restrict__ X, long n12, long nvox, ColTile ct,
                                                 const uint16_t* __restrict__ gmap, const T* __restrict__ Ctab,
                                                 T scale, const cplx<T>* __restrict__ tw,
                                                 const int* __restrict__ active, CellSel csel) {
  using V = cplx<T>;
  constexpr int NC = OP == 0 ? 6 : 3;
  constexpr int TP = TileCfg<T>::TP;
  constexpr int PPT = TP / NT;
  __shared__ V lds[TP];
  const int v = blockIdx.x / ct.tpv;
  const uint16_t* __restrict__ gmv = gmap + csel.goff(v);   // this vector's cell
  if (active && !active[v]) return;
  const int tile = blockIdx.x - v * ct.tpv;
  const int tid = threadIdx.x;
  const int line = tid & (ct.LT - 1);
  const long pos = (long)tile * ct.LT + line;
  const int npts = ct.LT * N0;
  V x[NC][PPT];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    cplx<T>* base = X + ((size_t)v * NC + c) * nvox + pos;
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int idx = tid + s * NT;
      if (idx < npts) {
        const int n = idx >> ct.lsh;
        lds[n * ct.LT + line] = base[(size_t)n * n12];
      }
    }
    __syncthreads();
    lds_fft<T, N0, true, NT, TP>(lds, ct.LT, ct.LT, ct.lsh, tw, tid);
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int idx = tid + s * NT;
      if (idx < npts) x[c][s] = lds[(idx >> ct.lsh) * ct.LT + line];
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int idx = tid + s * NT;
    if (idx < npts) {
      const int n = idx >> ct.lsh;
      const int g = gmv[(size_t)n * n12 + pos];
      if (OP == 0) {
        T cg[21];
#pragma unroll
        for (int i = 0; i < 21; ++i) cg[i] = Ctab[g * 21 + i];
        V e[6], sg[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) e[c] = x[c][s];
        contract6<T, V>(cg, e, sg, scale);
#pragma unroll
        for (int c = 0; c < 6; ++c) x[c][s] = sg[c];
      } else {
        const T rs = Ctab[g] * scale;
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c][s] = cscale(x[c][s], rs);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    cplx<T>* base = X + ((size_t)v * NC + c) * nvox + pos;
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int idx = tid + s * NT;
      if (idx < npts) lds[(idx >> ct.lsh) * ct.LT + line] = x[c][s];
    }
    __syncthreads();
    lds_fft<T, N0, false, NT, TP>(lds, ct.LT, ct.LT, ct.lsh, tw, tid);
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int idx = tid + s * NT;
      if (idx < npts) {
        const int n = idx >> ct.lsh;
        base[(size_t)n * n12] = lds[n * ct.LT + line];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// pointwise kernels over [nvec][3][nvox]; each block owns a chunk of voxels of
// one vector (grid = nvec * bpv).
// ---------------------------------------------------------------------------
// Flat voxel index -> (i0, i1, i2) in 32-bit arithmetic (a cell holds at most
// 2^30 voxels), with shifts and masks when n1 / n2 are powers of two (s1, s2 >= 0).
struct VoxIdx {
  int n0, n1, n2;
  int s1, s2;
  __device__ __forceinline__ void split(long vox, int& i0, int& i1, int& i2) const {
    const unsigned v = (unsigned)vox;
    unsigned r;
    if (s2 >= 0) {
      r = v >> s2;
      i2 = (int)(v & (unsigned)(n2 - 1));
    } else {
      r = v / (unsigned)n2;
      i2 = (int)(v - r * (unsigned)n2);
    }
    if (s1 >= 0) {
      i0 = (int)(r >> s1);
      i1 = (int)(r & (unsigned)(n1 - 1));
    } else {
      i0 = (int)(r / (unsigned)n1);
      i1 = (int)(r - (unsigned)i0 * (unsigned)n1);
    }
  }
};
inline int log2_exact(int n) {
  if (n <= 0 || (n & (n - 1))) return -1;
  int s = 0;
  while ((1 << s) < n) ++s;
  return s;
}
inline VoxIdx voxidx(const Geom& g) { return VoxIdx{g.n0, g.n1, g.n2, log2_exact(g.n1), log2_exact(g.n2)}; }

template <typename T>
__global__ __launch_bounds__(NT) void k_apply_P(const cplx<T>* __restrict__ U, cplx<T>* __restrict__ Y,
                                                const double* __restrict__ qtab, VoxIdx vi, long nvox, int bpv,
                                                C21v<T> C0, T scale, CellSel csel) {
  using V = cplx<T>;
  const int v = blockIdx.x / bpv;
  const int b = blockIdx.x - v * bpv;
  const double* q = qtab + (size_t)v * (vi.n0 + vi.n1 + vi.n2);
  const C21v<T> C0c = cell_c0<T>(csel, v, C0);
  for (long vox = (long)b * NT + threadIdx.x; vox < nvox; vox += (long)bpv * NT) {
    int i0, i1, i2;
    vi.split(vox, i0, i1, i2);
    V r[3], z[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = U[((size_t)v * 3 + c) * nvox + vox];
    precond3<T, V>(C0c, (T)q[i0], (T)q[vi.n0 + i1], (T)q[vi.n0 + vi.n1 + i2], r, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) Y[((size_t)v * 3 + c) * nvox + vox] = cscale(z[c], scale);
  }
}

// x += alpha p; r -= alpha Kp; z = P^ r; <r, z>, ||r||^2; last block: beta,
// convergence flag (recurrence residual below the threshold).
// WZ: also write z over K p (the next direction update reads it there).
template <typename T, bool WZ = false>
__global__ __launch_bounds__(NT) void k_pcg_update(cplx<T>* __restrict__ x, cplx<T>* __restrict__ r,
                                                   const cplx<T>* __restrict__ p, cplx<T>* __restrict__ Ap,
                                                   const double* __restrict__ qtab, VoxIdx vi, long nvox, int bpv,
                                                   C21v<T> C0, PcgDev pd, CellSel csel) {
  using V = cplx<T>;
  __shared__ double sh[NT / 64];
  const int v = blockIdx.x / bpv;
  const int b = blockIdx.x - v * bpv;
  if (!pd.active[v]) return;
  const T al = (T)pd.alpha[v];
  const double* q = qtab + (size_t)v * (vi.n0 + vi.n1 + vi.n2);
  const C21v<T> C0c = cell_c0<T>(csel, v, C0);
  double rz = 0, rr = 0;
  // this vector's arrays from uniform bases; component c of voxel vx at the 32-bit
  // offset c nvox + vx (3 nvox <= 3 2^30 < 2^32), so no 64-bit address is held
  // per access
  const size_t vb = (size_t)v * 3 * nvox;
  V* __restrict__ xb = x + vb;
  V* __restrict__ rb = r + vb;
  const V* __restrict__ pb = p + vb;
  V* __restrict__ ab = Ap + vb;
  const uint32_t n = (uint32_t)nvox;
  // two voxels of the thread's sequence per pass, all 24 loads issued before any
  // store (the same voxel order as one at a time, so the same sums)
  const uint32_t stride = (uint32_t)bpv * NT;
  for (uint32_t vox = (uint32_t)b * NT + threadIdx.x; vox < n; vox += 2 * stride) {
    const bool two = vox + stride < n;
    V pv[2][3], xv[2][3], rv[2][3], av[2][3];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      const uint32_t vx = vox + u * stride;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const uint32_t o = c * n + vx;
        pv[u][c] = pb[o];
        xv[u][c] = xb[o];
        rv[u][c] = rb[o];
        av[u][c] = ab[o];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      const uint32_t vx = vox + u * stride;
      int i0, i1, i2;
      vi.split(vx, i0, i1, i2);
      V z[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const uint32_t o = c * n + vx;
        xb[o] = caxpy(xv[u][c], al, pv[u][c]);
        rv[u][c] = caxpy(rv[u][c], -al, av[u][c]);
        rb[o] = rv[u][c];
      }
      precond3<T, V>(C0c, (T)q[i0], (T)q[vi.n0 + i1], (T)q[vi.n0 + vi.n1 + i2], rv[u], z);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        rz += (double)rv[u][c].x * z[c].x + (double)rv[u][c].y * z[c].y;
        rr += (double)rv[u][c].x * rv[u][c].x + (double)rv[u][c].y * rv[u][c].y;
        if (WZ) ab[c * n + vx] = z[c];
      }
    }
  }
  const double vals[2] = {rz, rr};
  store_partials<2>(vals, pd.partial, v, b, pd.max_blocks, sh);
}

// r = b - Kx (Kx given), ||r||^2 and ||b||^2 per vector (FP64).
template <typename T>
__global__ __launch_bounds__(NT) void k_residual(const cplx<T>* __restrict__ bv, const cplx<T>* __restrict__ Kx,
                                                 cplx<T>* __restrict__ r, long nvox3, int bpv, double* partial,
                                                 int maxb) {
  using V = cplx<T>;
  __shared__ double sh[NT / 64];
  const int v = blockIdx.x / bpv;
  const int b = blockIdx.x - v * bpv;
  double rr = 0, bb = 0;
  for (long i = (long)b * NT + threadIdx.x; i < nvox3; i += (long)bpv * NT) {
    const size_t o = (size_t)v * nvox3 + i;
    const V bb_ = bv[o];
    const V rv = Kx ? csub(bb_, Kx[o]) : bb_;
    r[o] = rv;
    rr += (double)rv.x * rv.x + (double)rv.y * rv.y;
    bb += (double)bb_.x * bb_.x + (double)bb_.y * bb_.y;
  }
  const double vals[2] = {rr, bb};
  store_partials<2>(vals, partial, v, b, maxb, sh);
}

// ||r||^2, ||b||^2 per vector of a given residual (read only)
template <typename T>
__global__ __launch_bounds__(NT) void k_norms2(const cplx<T>* __restrict__ bv, const cplx<T>* __restrict__ r,
                                               long nvox3, int bpv, double* partial, int maxb) {
  __shared__ double sh[NT / 64];
  const int v = blockIdx.x / bpv;
  const int b = blockIdx.x - v * bpv;
  double rr = 0, bb = 0;
  for (long i = (long)b * NT + threadIdx.x; i < nvox3; i += (long)bpv * NT) {
    const size_t o = (size_t)v * nvox3 + i;
    const cplx<T> rv = r[o], b_ = bv[o];
    rr += (double)rv.x * rv.x + (double)rv.y * rv.y;
    bb += (double)b_.x * b_.x + (double)b_.y * b_.y;
  }
  const double vals[2] = {rr, bb};
  store_partials<2>(vals, partial, v, b, maxb, sh);
}

// restart of the selected vectors: rz = <r, P^ r>, beta = 0
template <typename T>
__global__ __launch_bounds__(NT) void k_pcg_restart(const cplx<T>* __restrict__ r, const double* __restrict__ qtab,
                                                    VoxIdx vi, long nvox, int bpv, C21v<T> C0, PcgDev pd,
                                                    const int* __restrict__ mask, cplx<T>* __restrict__ zout,
                                                    CellSel csel) {
  using V = cplx<T>;
  __shared__ double sh[NT / 64];
  const int v = blockIdx.x / bpv;
  const int b = blockIdx.x - v * bpv;
  if (!mask[v]) return;
  const double* q = qtab + (size_t)v * (vi.n0 + vi.n1 + vi.n2);
  const C21v<T> C0c = cell_c0<T>(csel, v, C0);
  double rz = 0;
  for (long vox = (long)b * NT + threadIdx.x; vox < nvox; vox += (long)bpv * NT) {
    int i0, i1, i2;
    vi.split(vox, i0, i1, i2);
    V rv[3], z[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = r[((size_t)v * 3 + c) * nvox + vox];
    precond3<T, V>(C0c, (T)q[i0], (T)q[vi.n0 + i1], (T)q[vi.n0 + vi.n1 + i2], rv, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rz += (double)rv[c].x * z[c].x + (double)rv[c].y * z[c].y;
      if (zout) zout[((size_t)v * 3 + c) * nvox + vox] = z[c];
    }
  }
  const double vals[1] = {rz};
  store_partials<1>(vals, pd.partial, v, b, pd.max_blocks, sh);
}

// ---------------------------------------------------------------------------
// host-side tile selection and size dispatch
// ---------------------------------------------------------------------------
inline int ilog2(int x) {
  int l = 0;
  while ((1 << (l + 1)) <= x) ++l;
  return l;
}

template <typename T> RowTile row_tile(int N2, long rows_per_vec, int cap = 0) {
  constexpr int TP = TileCfg<T>::TP;
  int NR = 1;
  while (NR * 2 * N2 <= TP && rows_per_vec % (NR * 2) == 0 && (cap <= 0 || NR * 2 <= cap)) NR *= 2;
  return RowTile{NR, ilog2(NR), (int)(rows_per_vec / NR)};
}

template <typename T> ColTile axis1_tile(int N1, int n2, long lines_per_vec, int cap = 0) {
  constexpr int TP = TileCfg<T>::TP;
  int LT = 1;
  while (LT * 2 * N1 <= TP && LT * 2 <= NT && lines_per_vec % (LT * 2) == 0 &&
         (n2 % (LT * 2) == 0 || (LT * 2) % n2 == 0) && (cap <= 0 || LT * 2 <= cap))
    LT *= 2;
  return ColTile{LT, ilog2(LT), (int)(lines_per_vec / LT)};
}

template <typename T> ColTile axis0_tile(int N0, long n12, int cap = 0) {
  constexpr int TP = TileCfg<T>::TP;
  int LT = 1;
  while (LT * 2 * N0 <= TP && LT * 2 <= NT && n12 % (LT * 2) == 0 && (cap <= 0 || LT * 2 <= cap)) LT *= 2;
  return ColTile{LT, ilog2(LT), (int)(n12 / LT)};
}

#define BW_SIZES(X) X(1) X(2) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(40) X(48) X(64) X(96) X(128) X(256)

template <class F> void with_n(int n, F&& f) {
  switch (n) {
#define BW_CASE(N) \
  case N:          \
    f(std::integral_constant<int, N>{}); \
    break;
    BW_SIZES(BW_CASE)
#undef BW_CASE
    default:
      throw Error{BW_EUNSUPPORTED, "no compiled FFT of length " + std::to_string(n)};
  }
}

inline bool size_supported(int n) {
  switch (n) {
#define BW_CASE(N) case N:
    BW_SIZES(BW_CASE)
#undef BW_CASE
    return true;
    default:
      return false;
  }
}

template <typename T> const cplx<T>* twiddles(const bw_rve* r, int axis);
template <> inline const cplx<double>* twiddles<double>(const bw_rve* r, int axis) {
  return reinterpret_cast<const cplx<double>*>(r->d_tw64[axis]);
}
template <> inline const cplx<float>* twiddles<float>(const bw_rve* r, int axis) {
  return reinterpret_cast<const cplx<float>*>(r->d_tw32[axis]);
}
template <typename T> const T* ctab(const bw_rve* r);
template <> inline const double* ctab<double>(const bw_rve* r) { return r->d_C64; }
template <> inline const float* ctab<float>(const bw_rve* r) { return r->d_C32; }
template <typename T> const T* rhotab(const bw_rve* r);
template <> inline const double* rhotab<double>(const bw_rve* r) { return r->d_rho64; }
template <> inline const float* rhotab<float>(const bw_rve* r) { return r->d_rho32; }

template <typename T> C21v<T> c0v(const bw_rve* r) {
  C21v<T> c;
  for (int i = 0; i < 21; ++i) c.c[i] = (T)r->C0s[i];
  return c;
}

inline int pw_blocks(long nvox) {
  long b = (nvox + NT * 4 - 1) / (NT * 4);
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

}  // namespace bw
#include "bw_fftreg.h"
#include "bw_slab.h"
namespace bw {

// ---------------------------------------------------------------------------
// operator launchers
// ---------------------------------------------------------------------------
template <class F> void with_reg(int n, F&& f) {
  switch (n) {
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    default: throw Error{BW_EUNSUPPORTED, "no register FFT of length " + std::to_string(n)};
  }
}
template <typename T, int OP>
void launch_axis0(const bw_rve* r, cplx<T>* W, int nvec, T scale, const int* active, hipStream_t s,
                  const T* tab_override);

// Middle passes shared by K and M: inverse axis 1, axis-0 op, forward axis 1.
template <typename T, int OP>
void launch_middle(const bw_rve* r, cplx<T>* W, int nvec, T scale, const int* active, hipStream_t s,
                   const T* tab_override = nullptr) {
  const Geom& g = r->g;
  constexpr int NC = OP == 0 ? 6 : 3;
  const long n12 = (long)g.n1 * g.n2;
  const bool reg1 = r->tune_reg[tsel<T>][1] && reg_len(g.n1) && g.n2 % reg_lines(g.n1) == 0;
  auto axis1 = [&](auto INVc) {
    constexpr bool INV = decltype(INVc)::value;
    const char* name = active ? (INV ? "k_axis1_inv_pcg" : "k_axis1_fwd_pcg")
                              : (OP == 0 ? (INV ? "k_axis1_inv" : "k_axis1_fwd")
                                         : (INV ? "k_axis1_inv_mass" : "k_axis1_fwd_mass"));
    const long units = active ? 0 : nvec;
    if (reg1) {
      with_reg(g.n1, [&](auto N1) {
        constexpr int n1c = decltype(N1)::value;
        const int tpv = NC * g.n0 * (g.n2 / reg_lines(n1c));
        if (active)
          BW_LAUNCH(name, units, (k_axis1_r<T, n1c, INV, 1>), dim3(nvec * tpv), dim3(NT), 0, s, W, g.n2,
                    (long)NC * g.nvox, tpv, twiddles<T>(r, 1), active);
        else
          BW_LAUNCH(name, units, (k_axis1_r<T, n1c, INV, 0>), dim3(nvec * tpv), dim3(NT), 0, s, W, g.n2,
                    (long)NC * g.nvox, tpv, twiddles<T>(r, 1), active);
      });
      return;
    }
    with_n(g.n1, [&](auto N1) {
      ColTile ct = axis1_tile<T>(N1, g.n2, (long)NC * g.n0 * g.n2, r->tune_cap[tsel<T>][1]);
      if (active)
        BW_LAUNCH(name, units, (k_axis1<T, decltype(N1)::value, INV, 1>), dim3(nvec * ct.tpv), dim3(NT), 0, s, W,
                  g.n2, (long)NC * g.nvox, ct, twiddles<T>(r, 1), active);
      else
        BW_LAUNCH(name, units, (k_axis1<T, decltype(N1)::value, INV>), dim3(nvec * ct.tpv), dim3(NT), 0, s, W,
                  g.n2, (long)NC * g.nvox, ct, twiddles<T>(r, 1), active);
    });
  };
  if (g.n1 > 1) axis1(std::true_type{});
  launch_axis0<T, OP>(r, W, nvec, scale, active, s, tab_override);
  if (g.n1 > 1) axis1(std::false_type{});
}

// Axis-0 pass shared by K and M: inverse FFT along axis 0, pointwise op, forward FFT.
template <typename T, int OP>
void launch_axis0(const bw_rve* r, cplx<T>* W, int nvec, T scale, const int* active, hipStream_t s,
                  const T* tab_override) {
  const Geom& g = r->g;
  constexpr int NC = OP == 0 ? 6 : 3;
  const long n12 = (long)g.n1 * g.n2;
  const T* tab = tab_override ? tab_override : (OP == 0 ? ctab<T>(r) : rhotab<T>(r));
  const char* name0 = active ? "k_axis0_contract_pcg" : (OP == 0 ? "k_axis0_contract" : "k_axis0_mass");
  const long units0 = active ? 0 : nvec;
  if (r->tune_reg[tsel<T>][0] && reg_len(g.n0) && n12 % reg_lines(g.n0) == 0 && (long)NC * g.nvox < (1L << 31)) {
    with_reg(g.n0, [&](auto N0) {
      constexpr int n0c = decltype(N0)::value;
      const int tpv = (int)(n12 / reg_lines(n0c));
      if (active)
        BW_LAUNCH(name0, units0, (k_axis0_op_r<T, n0c, OP, 1>), dim3(nvec * tpv), dim3(NT), 0, s, W, n12, g.nvox,
                  tpv, r->d_gmap, tab, scale, twiddles<T>(r, 0), active, r->csel);
      else
        BW_LAUNCH(name0, units0, (k_axis0_op_r<T, n0c, OP, 0>), dim3(nvec * tpv), dim3(NT), 0, s, W, n12, g.nvox,
                  tpv, r->d_gmap, tab, scale, twiddles<T>(r, 0), active, r->csel);
    });
  } else {
    with_n(g.n0, [&](auto N0) {
      ColTile ct = axis0_tile<T>(N0, n12, r->tune_cap[tsel<T>][0]);
      if (active)
        BW_LAUNCH(name0, units0, (k_axis0_op<T, decltype(N0)::value, OP, 1>), dim3(nvec * ct.tpv), dim3(NT), 0, s,
                  W, n12, g.nvox, ct, r->d_gmap, tab, scale, twiddles<T>(r, 0), active, r->csel);
      else
        BW_LAUNCH(name0, units0, (k_axis0_op<T, decltype(N0)::value, OP>), dim3(nvec * ct.tpv), dim3(NT), 0, s, W,
                  n12, g.nvox, ct, r->d_gmap, tab, scale, twiddles<T>(r, 0), active, r->csel);
    });
  }
}

// The three-pass slab path (FP32, n1 = n2 = 128; bw_slab.h).  In PCG mode it takes
// the preconditioned residual z = P^ r from the K p buffer, where the update and
// restart kernels leave it.
template <typename T> inline bool slab_path(const bw_rve* r) {
  const Geom& g = r->g;
  return std::is_same<T, float>::value && r->tune_slab && g.n1 == SLAB_N && g.n2 == SLAB_N && g.n0 > 1 &&
         size_supported(g.n0) && 6L * g.nvox < (1L << 31);
}

template <typename T>
void apply_K_impl(const bw_rve* r, const double* d_qtab, const cplx<T>* u, cplx<T>* y, int nvec, double scale,
                  cplx<T>* W, hipStream_t s, int mode, cplx<T>* pp, const PcgDev* pd) {
  const Geom& g = r->g;
  const int* active = mode == 1 ? pd->active : nullptr;
  PcgDev dummy{};
  if constexpr (std::is_same<T, float>::value) {
    if (slab_path<T>(r)) {
      const dim3 grid(nvec * g.n0);
      const float2* tw = twiddles<T>(r, 2);
      if (mode == 0)
        BW_LAUNCH("k_slab_strain", nvec, (k_slab_strain<0>), grid, dim3(SLAB_NT), 0, s, u, (float2*)nullptr, W,
                  d_qtab, g.n0, g.nvox, tw, active, (const double*)nullptr);
      else   // u = r is not read: z = P^ r waits in y (the K p buffer)
        BW_LAUNCH("k_slab_strain_pcg", 0, (k_slab_strain<1>), grid, dim3(SLAB_NT), 0, s, (const float2*)y, pp, W,
                  d_qtab, g.n0, g.nvox, tw, active, pd->beta);
      launch_axis0<T, 0>(r, W, nvec, (T)(1.0 / (double)g.nvox), active, s, nullptr);
      if (mode == 0)
        BW_LAUNCH("k_slab_div", nvec, (k_slab_div<0>), grid, dim3(SLAB_NT), 0, s, (const float2*)W, y, d_qtab, g.n0,
                  g.nvox, tw, active, (const float2*)nullptr, dummy, (float)scale);
      else {
        BW_LAUNCH("k_slab_div_pcg", 0, (k_slab_div<1>), grid, dim3(SLAB_NT), 0, s, (const float2*)W, y, d_qtab,
                  g.n0, g.nvox, tw, active, (const float2*)pp, *pd, (float)scale);
        hipLaunchKernelGGL(k_finalize, dim3(nvec), dim3(NT), 0, s, (int)FIN_ALPHA, g.n0, *pd, (const int*)nullptr,
                           (double*)nullptr, (double*)nullptr);
      }
      return;
    }
  }
  const bool reg2 = r->tune_reg[tsel<T>][2] && reg_len(g.n2) && ((long)g.n0 * g.n1) % reg_lines(g.n2) == 0;
  const int tpvr = reg2 ? (int)(((long)g.n0 * g.n1) / reg_lines(g.n2)) : 0;
  // fused plane pass (FP32, n0 = n1 = 64): strain and stress in the transposed work layout
  const bool plane = std::is_same<T, float>::value && reg2 && r->tune_plane && r->d_gmapT && g.n0 == 64 &&
                     g.n1 == 64 && 6L * g.nvox < (1L << 31);
  if (reg2) {
    with_reg(g.n2, [&](auto N2) {
      constexpr int n2c = decltype(N2)::value;
      if (plane) {
        if (mode == 0)
          BW_LAUNCH("k_strain_row", nvec, (k_strain_row_r<T, n2c, 0, true>), dim3(nvec * tpvr), dim3(NT), 0, s, u,
                    (cplx<T>*)nullptr, W, d_qtab, g.n0, g.n1, g.nvox, tpvr, twiddles<T>(r, 2), active,
                    (const double*)nullptr, c0v<T>(r), r->csel);
        else
          BW_LAUNCH("k_strain_row_pcg", 0, (k_strain_row_r<T, n2c, 1, true>), dim3(nvec * tpvr), dim3(NT), 0, s, u,
                    pp, W, d_qtab, g.n0, g.n1, g.nvox, tpvr, twiddles<T>(r, 2), active, pd->beta, c0v<T>(r), r->csel);
      } else if (mode == 0)
        BW_LAUNCH("k_strain_row", nvec, (k_strain_row_r<T, n2c, 0>), dim3(nvec * tpvr), dim3(NT), 0, s, u,
                  (cplx<T>*)nullptr, W, d_qtab, g.n0, g.n1, g.nvox, tpvr, twiddles<T>(r, 2), active,
                  (const double*)nullptr, c0v<T>(r), r->csel);
      else
        BW_LAUNCH("k_strain_row_pcg", 0, (k_strain_row_r<T, n2c, 1>), dim3(nvec * tpvr), dim3(NT), 0, s, u, pp, W,
                  d_qtab, g.n0, g.n1, g.nvox, tpvr, twiddles<T>(r, 2), active, pd->beta, c0v<T>(r), r->csel);
    });
  } else {
    with_n(g.n2, [&](auto N2) {
      constexpr int n2c = decltype(N2)::value;
      RowTile rt = row_tile<T>(n2c, (long)g.n0 * g.n1, r->tune_cap[tsel<T>][2]);
      if (mode == 0)
        BW_LAUNCH("k_strain_row", nvec, (k_strain_row<T, n2c, 0>), dim3(nvec * rt.tpv), dim3(NT), 0, s, u,
                  (cplx<T>*)nullptr, W, d_qtab, g.n0, g.n1, g.nvox, rt, twiddles<T>(r, 2), active,
                  (const double*)nullptr, c0v<T>(r), r->csel);
      else
        BW_LAUNCH("k_strain_row_pcg", 0, (k_strain_row<T, n2c, 1>), dim3(nvec * rt.tpv), dim3(NT), 0, s, u, pp, W,
                  d_qtab, g.n0, g.n1, g.nvox, rt, twiddles<T>(r, 2), active, pd->beta, c0v<T>(r), r->csel);
    });
  }
  if (plane) {
    if constexpr (std::is_same<T, float>::value) {   // the plane kernel exists for FP32 only
      // persistent: one workgroup per CU (the kernel's LDS and registers admit one)
      const int nplanes = nvec * g.n2;
      const int grid = std::min(nplanes, std::max(r->ncu, 1));
      const T sc = (T)(1.0 / (double)g.nvox);
      const bool cl = r->G <= PLANE_CL_MAX;
      if (active) {
        if (cl)
          BW_LAUNCH("k_plane_contract_pcg", 0, (k_plane64<T, 1, true>), dim3(grid), dim3(PLANE_NT), 0, s, W, g.n2,
                    nplanes, g.nvox, r->d_gmapT, ctab<T>(r), r->G, sc, twiddles<T>(r, 0), active,
                    r->csel);
        else
          BW_LAUNCH("k_plane_contract_pcg", 0, (k_plane64<T, 1, false>), dim3(grid), dim3(PLANE_NT), 0, s, W, g.n2,
                    nplanes, g.nvox, r->d_gmapT, ctab<T>(r), r->G, sc, twiddles<T>(r, 0), active,
                    r->csel);
      } else {
        if (cl)
          BW_LAUNCH("k_plane_contract", nvec, (k_plane64<T, 0, true>), dim3(grid), dim3(PLANE_NT), 0, s, W, g.n2,
                    nplanes, g.nvox, r->d_gmapT, ctab<T>(r), r->G, sc, twiddles<T>(r, 0), active,
                    r->csel);
        else
          BW_LAUNCH("k_plane_contract", nvec, (k_plane64<T, 0, false>), dim3(grid), dim3(PLANE_NT), 0, s, W, g.n2,
                    nplanes, g.nvox, r->d_gmapT, ctab<T>(r), r->G, sc, twiddles<T>(r, 0), active,
                    r->csel);
      }
    }
  } else {
    launch_middle<T, 0>(r, W, nvec, (T)(1.0 / (double)g.nvox), active, s);
  }
  int nblk = 0;
  if (reg2) {
    nblk = tpvr;
    with_reg(g.n2, [&](auto N2) {
      constexpr int n2c = decltype(N2)::value;
      if (plane) {
        if (mode == 0)
          BW_LAUNCH("k_row_div", nvec, (k_row_div_r<T, n2c, 0, true>), dim3(nvec * tpvr), dim3(NT), 0, s, W, y,
                    d_qtab, g.n0, g.n1, g.nvox, tpvr, twiddles<T>(r, 2), active, (const cplx<T>*)nullptr, dummy,
                    (T)scale);
        else
          BW_LAUNCH("k_row_div_pcg", 0, (k_row_div_r<T, n2c, 1, true>), dim3(nvec * tpvr), dim3(NT), 0, s, W, y,
                    d_qtab, g.n0, g.n1, g.nvox, tpvr, twiddles<T>(r, 2), active, (const cplx<T>*)pp, *pd, (T)scale);
        return;
      }
      if (mode == 0)
        BW_LAUNCH("k_row_div", nvec, (k_row_div_r<T, n2c, 0>), dim3(nvec * tpvr), dim3(NT), 0, s, W, y, d_qtab,
                  g.n0, g.n1, g.nvox, tpvr, twiddles<T>(r, 2), active, (const cplx<T>*)nullptr, dummy, (T)scale);
      else
        BW_LAUNCH("k_row_div_pcg", 0, (k_row_div_r<T, n2c, 1>), dim3(nvec * tpvr), dim3(NT), 0, s, W, y, d_qtab,
                  g.n0, g.n1, g.nvox, tpvr, twiddles<T>(r, 2), active, (const cplx<T>*)pp, *pd, (T)scale);
    });
  } else {
    with_n(g.n2, [&](auto N2) {
      constexpr int n2c = decltype(N2)::value;
      RowTile rt = row_tile<T>(n2c, (long)g.n0 * g.n1, r->tune_cap[tsel<T>][2]);
      nblk = rt.tpv;
      if (mode == 0)
        BW_LAUNCH("k_row_div", nvec, (k_row_div<T, n2c, 0>), dim3(nvec * rt.tpv), dim3(NT), 0, s, W, y, d_qtab,
                  g.n0, g.n1, g.nvox, rt, twiddles<T>(r, 2), active, (const cplx<T>*)nullptr, dummy, (T)scale);
      else
        BW_LAUNCH("k_row_div_pcg", 0, (k_row_div<T, n2c, 1>), dim3(nvec * rt.tpv), dim3(NT), 0, s, W, y, d_qtab,
                  g.n0, g.n1, g.nvox, rt, twiddles<T>(r, 2), active, (const cplx<T>*)pp, *pd, (T)scale);
    });
  }
  if (mode == 1)
    hipLaunchKernelGGL(k_finalize, dim3(nvec), dim3(NT), 0, s, (int)FIN_ALPHA, nblk, *pd, (const int*)nullptr,
                       (double*)nullptr, (double*)nullptr);
}

template <typename T>
void launch_apply_K(const bw_rve* r, const double* d_qtab, const cplx<T>* u, cplx<T>* y, int nvec, double scale,
                    cplx<T>* W, hipStream_t s) {
  apply_K_impl<T>(r, d_qtab, u, y, nvec, scale, W, s, 0, nullptr, nullptr);
}

template <typename T> const T* rhoinvtab(const bw_rve* r);
template <> inline const double* rhoinvtab<double>(const bw_rve* r) { return r->d_rhoinv64; }
template <> inline const float* rhoinvtab<float>(const bw_rve* r) { return r->d_rhoinv32; }

template <typename T>
void apply_M_impl(const bw_rve* r, const cplx<T>* u, cplx<T>* y, int nvec, double scale, cplx<T>* W, hipStream_t s,
                  const T* tab) {
  const Geom& g = r->g;
  const long rows = 3L * g.n0 * g.n1;
  with_n(g.n2, [&](auto N2) {
    constexpr int n2c = decltype(N2)::value;
    RowTile rt = row_tile<T>(n2c, rows, r->tune_cap[tsel<T>][2]);
    BW_LAUNCH("k_row_inv_mass", nvec, (k_row_plain<T, n2c, true>), dim3(nvec * rt.tpv), dim3(NT), 0, s, u, W, rt,
              (int)rows,
                       twiddles<T>(r, 2), (const int*)nullptr);
  });
  launch_middle<T, 1>(r, W, nvec, (T)(scale / (double)g.nvox), nullptr, s, tab);
  with_n(g.n2, [&](auto N2) {
    constexpr int n2c = decltype(N2)::value;
    RowTile rt = row_tile<T>(n2c, rows, r->tune_cap[tsel<T>][2]);
    BW_LAUNCH("k_row_fwd_mass", nvec, (k_row_plain<T, n2c, false>), dim3(nvec * rt.tpv), dim3(NT), 0, s,
              (const cplx<T>*)W, y, rt,
                       (int)rows, twiddles<T>(r, 2), (const int*)nullptr);
  });
}

template <typename T>
void launch_apply_M(const bw_rve* r, const cplx<T>* u, cplx<T>* y, int nvec, double scale, cplx<T>* W,
                    hipStream_t s) {
  apply_M_impl<T>(r, u, y, nvec, scale, W, s, nullptr);
}

template <typename T>
void launch_apply_Minv_or_M(const bw_rve* r, const cplx<T>* u, cplx<T>* y, int nvec, bool inverse, cplx<T>* W,
                            hipStream_t s) {
  apply_M_impl<T>(r, u, y, nvec, 1.0, W, s, inverse ? rhoinvtab<T>(r) : rhotab<T>(r));
}

template <typename T>
void launch_apply_P(const bw_rve* r, const double* d_qtab, const cplx<T>* u, cplx<T>* y, int nvec, double scale,
                    hipStream_t s) {
  const Geom& g = r->g;
  const int bpv = pw_blocks(g.nvox);
  hipLaunchKernelGGL((k_apply_P<T>), dim3(nvec * bpv), dim3(NT), 0, s, u, y, d_qtab, voxidx(g),
                     g.nvox, bpv, c0v<T>(r), (T)scale, r->csel);
}

template <typename T>
void launch_pcg_apply(const bw_rve* r, const double* d_qtab, const cplx<T>* rv, cplx<T>* p, cplx<T>* Ap, cplx<T>* W,
                      int nvec, const PcgDev& pd, hipStream_t s) {
  apply_K_impl<T>(r, d_qtab, rv, Ap, nvec, 1.0, W, s, 1, p, &pd);
}

template <typename T>
void launch_pcg_update(const bw_rve* r, const double* d_qtab, cplx<T>* x, cplx<T>* rv, const cplx<T>* p,
                       cplx<T>* Ap, int nvec, const PcgDev& pd, hipStream_t s) {
  const Geom& g = r->g;
  const int bpv = pw_blocks(g.nvox);
  if (slab_path<T>(r))
    BW_LAUNCH("k_pcg_update_z", 0, (k_pcg_update<T, true>), dim3(nvec * bpv), dim3(NT), 0, s, x, rv, p, Ap, d_qtab,
              voxidx(g), g.nvox, bpv, c0v<T>(r), pd, r->csel);
  else
    BW_LAUNCH("k_pcg_update", 0, (k_pcg_update<T>), dim3(nvec * bpv), dim3(NT), 0, s, x, rv, p, Ap, d_qtab,
              voxidx(g), g.nvox, bpv, c0v<T>(r), pd, r->csel);
  hipLaunchKernelGGL(k_finalize, dim3(nvec), dim3(NT), 0, s, (int)FIN_BETA, bpv, pd, (const int*)nullptr,
                     (double*)nullptr, (double*)nullptr);
}

template <typename T>
void launch_residual(const bw_rve* r, const double* d_qtab, const cplx<T>* b, const cplx<T>* x, cplx<T>* rv,
                     cplx<T>* tmp, cplx<T>* W, int nvec, double* d_rr, double* d_bb, double* d_partial,
                     unsigned* d_counter, int max_blocks, hipStream_t s) {
  const Geom& g = r->g;
  if (x) launch_apply_K<T>(r, d_qtab, x, tmp, nvec, 1.0, W, s);
  const int bpv = pw_blocks(g.nvox * 3);
  hipLaunchKernelGGL((k_residual<T>), dim3(nvec * bpv), dim3(NT), 0, s, b, x ? (const cplx<T>*)tmp : nullptr, rv,
                     g.nvox * 3, bpv, d_partial, max_blocks);
  PcgDev pd{};
  pd.partial = d_partial;
  pd.max_blocks = max_blocks;
  hipLaunchKernelGGL(k_finalize, dim3(nvec), dim3(NT), 0, s, (int)FIN_RESID, bpv, pd, (const int*)nullptr, d_rr,
                     d_bb);
}

template <typename T>
void launch_norms2(const bw_rve* r, const cplx<T>* b, const cplx<T>* rv, int nvec, double* d_rr, double* d_bb,
                   double* d_partial, int max_blocks, hipStream_t s) {
  const Geom& g = r->g;
  const int bpv = pw_blocks(g.nvox * 3);
  hipLaunchKernelGGL((k_norms2<T>), dim3(nvec * bpv), dim3(NT), 0, s, b, rv, g.nvox * 3, bpv, d_partial, max_blocks);
  PcgDev pd{};
  pd.partial = d_partial;
  pd.max_blocks = max_blocks;
  hipLaunchKernelGGL(k_finalize, dim3(nvec), dim3(NT), 0, s, (int)FIN_RESID, bpv, pd, (const int*)nullptr, d_rr,
                     d_bb);
}

template <typename T>
void launch_pcg_restart(const bw_rve* r, const double* d_qtab, const cplx<T>* rv, int nvec, const PcgDev& pd,
                        const int* d_mask, hipStream_t s, cplx<T>* Ap) {
  const Geom& g = r->g;
  const int bpv = pw_blocks(g.nvox);
  hipLaunchKernelGGL((k_pcg_restart<T>), dim3(nvec * bpv), dim3(NT), 0, s, rv, d_qtab, voxidx(g),
                     g.nvox, bpv, c0v<T>(r), pd, d_mask, slab_path<T>(r) ? Ap : (cplx<T>*)nullptr,
                     r->csel);
  hipLaunchKernelGGL(k_finalize, dim3(nvec), dim3(NT), 0, s, (int)FIN_RESTART, bpv, pd, d_mask, (double*)nullptr,
                     (double*)nullptr);
}

template <typename T>
__global__ void k_scale(cplx<T>* x, size_t n, T sc) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = cscale(x[i], sc);
}
template <typename T>
__global__ void k_zero_voxel(cplx<T>* x, int nvec, long nvox, long vox) {
  const int i = threadIdx.x;
  if (i < nvec * 3) x[(size_t)i * nvox + vox] = cplx<T>{0, 0};
}
template <typename T> void scale_vectors(cplx<T>* x, size_t n, double sc, hipStream_t s) {
  if (n == 0) return;
  long b = (long)((n + NT - 1) / NT);
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL((k_scale<T>), dim3((unsigned)b), dim3(NT), 0, s, x, n, (T)sc);
}
template <typename T> void zero_voxel(cplx<T>* x, int nvec, long nvox, long vox, hipStream_t s) {
  for (int v0 = 0; v0 < nvec; v0 += 64) {
    const int nv = nvec - v0 < 64 ? nvec - v0 : 64;
    hipLaunchKernelGGL((k_zero_voxel<T>), dim3(1), dim3(192), 0, s, x + (size_t)v0 * 3 * nvox, nv, nvox, vox);
  }
}

#define BW_INSTANTIATE_OPS(T)                                                                                      \
  template void launch_apply_K<T>(const bw_rve*, const double*, const cplx<T>*, cplx<T>*, int, double, cplx<T>*,    \
                                  hipStream_t);                                                                    \
  template void launch_apply_M<T>(const bw_rve*, const cplx<T>*, cplx<T>*, int, double, cplx<T>*, hipStream_t);     \
  template void launch_apply_Minv_or_M<T>(const bw_rve*, const cplx<T>*, cplx<T>*, int, bool, cplx<T>*, hipStream_t); \
  template void launch_apply_P<T>(const bw_rve*, const double*, const cplx<T>*, cplx<T>*, int, double, hipStream_t); \
  template void launch_pcg_apply<T>(const bw_rve*, const double*, const cplx<T>*, cplx<T>*, cplx<T>*, cplx<T>*,     \
                                    int, const PcgDev&, hipStream_t);                                              \
  template void launch_pcg_update<T>(const bw_rve*, const double*, cplx<T>*, cplx<T>*, const cplx<T>*,              \
                                     cplx<T>*, int, const PcgDev&, hipStream_t);                                   \
  template void launch_residual<T>(const bw_rve*, const double*, const cplx<T>*, const cplx<T>*, cplx<T>*,          \
                                   cplx<T>*, cplx<T>*, int, double*, double*, double*, unsigned*, int, hipStream_t); \
  template void launch_pcg_restart<T>(const bw_rve*, const double*, const cplx<T>*, int, const PcgDev&, const int*, \
                                      hipStream_t, cplx<T>*);                                                       \
  template void launch_norms2<T>(const bw_rve*, const cplx<T>*, const cplx<T>*, int, double*, double*, double*, int, \
                                 hipStream_t);                                                                      \
  template void scale_vectors<T>(cplx<T>*, size_t, double, hipStream_t);                                           \
  template void zero_voxel<T>(cplx<T>*, int, long, long, hipStream_t);

}  // namespace bw
