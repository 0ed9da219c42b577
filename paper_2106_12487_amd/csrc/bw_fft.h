// Device building blocks: complex arithmetic and a Stockham autosort FFT that
// runs on a tile of lines held in LDS.
//
// Tile layout in LDS: element (point n, line l) at buf[n * P + l]; the FFT is
// taken along n for every line l < lines.  `lines` is a power of two
// (lshift = log2(lines)); P >= lines is the row pitch.  Every thread of the
// workgroup takes part.  Each radix-R pass reads its butterflies into
// registers, synchronizes, and writes them back in place, so one buffer is
// enough.  The forward transform uses exp(-2 pi i / N), the inverse one
// exp(+2 pi i / N); neither is scaled.
//
// Twiddles come from a table tw[t] = exp(-2 pi i t / N), t < N, computed on the
// host in double precision (and rounded once for the float table).
#pragma once
#include <hip/hip_runtime.h>

namespace bw {

template <typename T> struct cx_t;
template <> struct cx_t<float> { using type = float2; };
template <> struct cx_t<double> { using type = double2; };
template <typename T> using cplx = typename cx_t<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
  return V{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { return V{a.x * s, a.y * s}; }
// a + s * b with real s
template <typename V, typename S> __device__ __forceinline__ V caxpy(V a, S s, V b) {
  return V{a.x + s * b.x, a.y + s * b.y};
}
// (sign * i) * a with sign = +1 for the inverse transform, -1 for the forward one
template <bool INV, typename V> __device__ __forceinline__ V mul_si(V a) {
  return INV ? V{-a.y, a.x} : V{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// small DFTs of length R on registers: y_k = sum_n x_n exp(s 2 pi i n k / R)
// ---------------------------------------------------------------------------
template <int R, bool INV, typename V> struct SmallDFT;

template <bool INV, typename V> struct SmallDFT<2, INV, V> {
  __device__ __forceinline__ static void run(V* v) {
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV, typename V> struct SmallDFT<4, INV, V> {
  __device__ __forceinline__ static void run(V* v) {
    V t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    V t2 = cadd(v[1], v[3]), t3 = mul_si<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <bool INV, typename V> struct SmallDFT<8, INV, V> {
  __device__ __forceinline__ static void run(V* v) {
    using S = decltype(v[0].x);
    const S h = S(0.70710678118654752440084436210485);
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    SmallDFT<4, INV, V>::run(e);
    SmallDFT<4, INV, V>::run(o);
    // w^1 = h (1 + s i), w^2 = s i, w^3 = h (-1 + s i)
    V o1 = cscale(cadd(o[1], mul_si<INV>(o[1])), h);
    V o2 = mul_si<INV>(o[2]);
    V o3 = cscale(csub(mul_si<INV>(o[3]), o[3]), h);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <bool INV, typename V> struct SmallDFT<3, INV, V> {
  __device__ __forceinline__ static void run(V* v) {
    using S = decltype(v[0].x);
    const S c = S(-0.5), s3 = S(0.86602540378443864676372317075294);
    V a = cadd(v[1], v[2]), b = csub(v[1], v[2]);
    V m = caxpy(v[0], c, a);
    V t = cscale(mul_si<INV>(b), s3);
    v[0] = cadd(v[0], a);
    v[1] = cadd(m, t);
    v[2] = csub(m, t);
  }
};

template <bool INV, typename V> struct SmallDFT<5, INV, V> {
  __device__ __forceinline__ static void run(V* v) {
    using S = decltype(v[0].x);
    const S c1 = S(0.30901699437494742410229341718282), c2 = S(-0.80901699437494742410229341718282);
    const S s1 = S(0.95105651629515357211643933337938), s2 = S(0.58778525229247312916870595463907);
    V a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    V a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    V m1 = caxpy(caxpy(v[0], c1, a1), c2, a2);
    V m2 = caxpy(caxpy(v[0], c2, a1), c1, a2);
    V t1 = mul_si<INV>(V{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    V t2 = mul_si<INV>(V{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(m1, t1);
    v[4] = csub(m1, t1);
    v[2] = cadd(m2, t2);
    v[3] = csub(m2, t2);
  }
};

constexpr int pick_radix(int rem) {
  return rem == 16 ? 4 : (rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : (rem % 2 == 0 ? 2 : (rem % 3 == 0 ? 3 : (rem % 5 == 0 ? 5 : rem)))));
}

constexpr bool fft_length_ok(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}

// One radix-R pass of the Stockham algorithm (span NS before the pass).
template <typename T, int N, int R, int NS, bool INV, int NT, int TP>
__device__ __forceinline__ void stockham_pass(cplx<T>* buf, int P, int lines, int lshift,
                                              const cplx<T>* __restrict__ tw, int tid) {
  using V = cplx<T>;
  constexpr int NBL = N / R;                 // butterflies per line
  constexpr int NBT = (TP / R + NT - 1) / NT;  // butterflies per thread (upper bound)
  const int nb = NBL << lshift;
  V v[NBT][R];
#pragma unroll
  for (int t = 0; t < NBT; ++t) {
    const int b = tid + t * NT;
    if (b < nb) {
      const int line = b & (lines - 1);
      const int j = b >> lshift;
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = buf[(j + r * NBL) * P + line];
      if (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V w = tw[r * k * (N / (NS * R))];
          v[t][r] = INV ? cmulc(v[t][r], w) : cmul(v[t][r], w);
        }
      }
      SmallDFT<R, INV, V>::run(v[t]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < NBT; ++t) {
    const int b = tid + t * NT;
    if (b < nb) {
      const int line = b & (lines - 1);
      const int j = b >> lshift;
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(base + r * NS) * P + line] = v[t][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int NS, bool INV, int NT, int TP>
__device__ __forceinline__ void fft_passes(cplx<T>* buf, int P, int lines, int lshift,
                                           const cplx<T>* __restrict__ tw, int tid) {
  if constexpr (NS < N) {
    constexpr int R = pick_radix(N / NS);
    static_assert(R == 2 || R == 3 || R == 4 || R == 5 || R == 8, "FFT length must be 2^a 3^b 5^c");
    stockham_pass<T, N, R, NS, INV, NT, TP>(buf, P, lines, lshift, tw, tid);
    fft_passes<T, N, NS * R, INV, NT, TP>(buf, P, lines, lshift, tw, tid);
  }
}

// FFT of every line of the LDS tile (caller synchronizes before the call; the
// call ends with a barrier).
template <typename T, int N, bool INV, int NT, int TP>
__device__ __forceinline__ void lds_fft(cplx<T>* buf, int P, int lines, int lshift,
                                        const cplx<T>* __restrict__ tw, int tid) {
  fft_passes<T, N, 1, INV, NT, TP>(buf, P, lines, lshift, tw, tid);
}

}  // namespace bw
