// bw_apply_K_noalloc: the K operator (Sec. 3.2 eq. hatA) without any device
// allocation, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops).  The strain / stress work array and the wave-number
// table live in `scratch`, a fixed area of the library in each device's
// memory; the kernels are those of bw_apply_K.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "bw_internal.h"

namespace bw {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

// Host code must not use this name as a device address: kernels get the
// per-device address obtained below with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The address of this device's copy of `scratch` (looked up once per device,
// with that device current).
static void* scratch_ptr() {
  int dev = 0;
  BW_HIP(hipGetDevice(&dev));
  BW_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, BW_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    BW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BW_REQUIRE(p != nullptr, BW_EHIP, "hipGetSymbolAddress returned no address for the scratch area");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Per-axis data of the shifted wave numbers: q_a(j) = (2 pi m / L_a + k_a) ell
// with m = lo + ((j - lo) mod n_a); the same expression and order as the host
// table of the other entry points, so the values are identical.
struct QAxes {
  int n[3];
  int lo[3];
  double k[3];
  double L[3];
  double ell;
};

static __global__ void k_qrows(double* __restrict__ q, int nvec, QAxes ax) {
  const int per = ax.n[0] + ax.n[1] + ax.n[2];
  const long total = (long)nvec * per;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    int e = (int)(i % per);
    int a = 0;
    while (e >= ax.n[a]) e -= ax.n[a++];
    int mm = (e - ax.lo[a]) % ax.n[a];
    if (mm < 0) mm += ax.n[a];
    const int m = ax.lo[a] + mm;
    const double qv = 2.0 * M_PI * m / ax.L[a] + ax.k[a];
    q[i] = qv * ax.ell;
  }
}

}  // namespace bw

using namespace bw;

extern "C" int bw_apply_K_noalloc(bw_rve* r, const double k[3], const void* u, void* y, int32_t nvec,
                                  void* stream) {
  try {
    BW_REQUIRE(r && k, BW_EINVAL, "null argument");
    BW_REQUIRE(nvec >= 0, BW_EINVAL, "nvec < 0");
    if (nvec == 0) return BW_OK;
    BW_REQUIRE(u && y, BW_EINVAL, "null argument");
    BW_REQUIRE(u != y, BW_EINVAL, "u and y must not alias");
    const Geom& g = r->g;
    const size_t word = r->precision == BW_FP64 ? 16 : 8;
    const size_t wbytes = ((size_t)nvec * 6 * g.nvox * word + 255) / 256 * 256;
    const size_t qbytes = (size_t)nvec * (g.n0 + g.n1 + g.n2) * sizeof(double);
    BW_REQUIRE(wbytes + qbytes <= NOALLOC_SCRATCH_BYTES, BW_EINVAL,
               "bw_apply_K_noalloc: nvec * 6 * n0 n1 n2 complex words (" + std::to_string(wbytes + qbytes) +
                   " bytes with the wave-number table) exceed the scratch area of " +
                   std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes");
    char* base = (char*)scratch_ptr();   // the current device's copy (the cell's device, as for bw_apply_K)
    hipStream_t s = (hipStream_t)stream;
    // the wave-number table, written on the device (no host copy)
    QAxes ax{};
    const int n[3] = {g.n0, g.n1, g.n2};
    for (int a = 0; a < 3; ++a) {
      double ka = k[a];
      const double kappa = ka * r->L[a] / (2.0 * M_PI);
      const double gq = std::nearbyint(kappa);
      double kap = kappa;
      if (std::fabs(kappa - gq) <= 1e-9) {   // snapped to the reciprocal vector, as the host table
        kap = gq;
        ka = 2.0 * M_PI * gq / r->L[a];
      }
      ax.n[a] = n[a];
      ax.lo[a] = -(n[a] / 2) - (int)std::ceil(kap - 0.5 - 1e-9);
      ax.k[a] = ka;
      ax.L[a] = r->L[a];
    }
    ax.ell = r->ell;
    double* q = (double*)(base + wbytes);
    const long total = (long)nvec * (g.n0 + g.n1 + g.n2);
    const int blocks = (int)std::min<long>((total + 255) / 256, 1024);
    hipLaunchKernelGGL(k_qrows, dim3(blocks), dim3(256), 0, s, q, nvec, ax);
    if (r->precision == BW_FP64)
      launch_apply_K<double>(r, q, (const cplx<double>*)u, (cplx<double>*)y, nvec, K_scale(r), (cplx<double>*)base,
                             s);
    else
      launch_apply_K<float>(r, q, (const cplx<float>*)u, (cplx<float>*)y, nvec, K_scale(r), (cplx<float>*)base, s);
    BW_HIP(hipGetLastError());
    return BW_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal: ") + e.what());
    return BW_EINVAL;
  }
}
