// Internal declarations shared by the translation units of libblochwave.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/blochwave.h"
#include "bw_fft.h"

namespace bw {

constexpr int NT = 256;  // threads per workgroup of the FFT / pointwise kernels

// Maximum tile points per workgroup (one component of a tile is staged in LDS;
// all components of a point live in registers).
template <typename T> struct TileCfg;
template <> struct TileCfg<float> { static constexpr int TP = 2048; };
template <> struct TileCfg<double> { static constexpr int TP = 1024; };

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
struct Error {
  int code;
  std::string msg;
};
#define BW_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::bw::Error{BW_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)};      \
  } while (0)
#define BW_REQUIRE(cond, code, msg)                   \
  do {                                                \
    if (!(cond)) throw ::bw::Error{(code), (msg)};    \
  } while (0)

// ---------------------------------------------------------------------------
// opt-in kernel timing: HIP events around each launch, totals per kernel name
// (name, launches, milliseconds, work units = vectors processed)
// ---------------------------------------------------------------------------
bool timing_enabled();
bool graphs_enabled();
struct KTimer {
  const char* name;
  hipStream_t s;
  long units;
  hipEvent_t e0 = nullptr;
  KTimer(const char* n, hipStream_t st, long u);
  ~KTimer();
};
void timing_add_units(const char* name, long units);
#define BW_LAUNCH(name, units, kern, grid, block, shm, s, ...)  \
  do {                                                         \
    ::bw::KTimer kt_((name), (s), (units));                    \
    hipLaunchKernelGGL(kern, grid, block, shm, s, __VA_ARGS__); \
  } while (0)

// Device allocation and freeing (hipFree synchronizes the device) must not
// overlap a stream capture on another host thread: both hold this mutex.
std::recursive_mutex& capture_alloc_mutex();

// ---------------------------------------------------------------------------
// device buffer with grow-on-demand semantics
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void* get(size_t need) {
    if (need > bytes) {
      std::lock_guard<std::recursive_mutex> lk(capture_alloc_mutex());
      if (p) BW_HIP(hipFree(p));
      p = nullptr;
      bytes = 0;
      hipError_t e = hipMalloc(&p, need);
      if (e != hipSuccess) throw Error{BW_ENOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed"};
      bytes = need;
    }
    return p;
  }
  void release() {
    if (!p) return;
    std::lock_guard<std::recursive_mutex> lk(capture_alloc_mutex());
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Host-to-device copy of a host buffer that the caller may change or free as
// soon as this returns: a copy from pageable memory may read the host buffer
// only when it executes on the stream, so the stream is synchronized first.
inline void h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  BW_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
  BW_HIP(hipStreamSynchronize(s));
}

// Bloch data of a batch: per vector the scaled shifted wavevector tables
// q_a(j) = m_a(j) L0 / L_a + k_a L0 / (2 pi), concatenated [n0 | n1 | n2].
struct QTable {
  std::vector<double> host;   // nvec * (n0 + n1 + n2)
  int nvec = 0;
  std::vector<int> null_index;  // per vector: flat voxel index where q = 0, or -1
};

// Geometry and per-launch tile choices of one cell.
// Cells of one grid solved as one batch (bw_lowest_modes_batched): vector v of a
// launch belongs to cell(v) = the number of bounds <= v; that cell's grain map
// starts at cell * gstride and its reference stiffness C0 (scaled, 21 entries) is
// row `cell` of c0tab32 / c0tab64.  n = 1 (the default): one cell, the kernels'
// own C0 and grain map.
constexpr int CELLS_MAX = 8;
struct CellSel {
  int n = 1;
  int bound[CELLS_MAX - 1] = {};
  long gstride = 0;
  const float* c0tab32 = nullptr;
  const double* c0tab64 = nullptr;
  __host__ __device__ int cell(int v) const {
    int c = 0;
    for (int i = 0; i + 1 < n; ++i) c += v >= bound[i] ? 1 : 0;
    return c;
  }
  __host__ __device__ long goff(int v) const { return n > 1 ? (long)cell(v) * gstride : 0; }
};

struct Geom {
  int n0, n1, n2;
  long nvox;
};

// Cached vector workspaces of one precision.
template <typename T> struct Workspace {
  DevBuf v[16];
  DevBuf w;
  cplx<T>* vec(int i, size_t n) { return (cplx<T>*)v[i].get(n * sizeof(cplx<T>)); }
  cplx<T>* work(size_t n) { return (cplx<T>*)w.get(n * sizeof(cplx<T>)); }
  void release() {
    for (auto& b : v) b.release();
    w.release();
  }
};

struct PcgResult {
  std::vector<int> iters;
  std::vector<double> relres;
  bool converged = false;
  long total_iters = 0;
  long block_iters = 0;
  long k_applies = 0;  // single-vector K applies, residual checks included
};

}  // namespace bw

// The opaque cell handle.
struct bw_rve {
  bw::Geom g;
  double L[3];
  int G;
  int precision;
  int device;
  int ncu = 0;      // compute units of the device (persistent launches)
  // nondimensionalization: C' = C / Cref, q' = q * ell, rho' = rho / rho_bar
  double Cref, ell, rho_bar;
  double rho_min_s;  // smallest scaled density (bounds the M^-1 norm)
  int rho_unit = 0;  // every occupied grain has the mean density: M' = identity
  double C0_si[21];     // volume-averaged stiffness (Pa)
  double C0s[21];       // scaled
  std::vector<double> C21s_host;  // G x 21 scaled
  std::vector<double> rhos_host;  // G scaled
  std::vector<uint16_t> gmap_host;
  // device copies
  uint16_t* d_gmap = nullptr;
  uint16_t* d_gmapT = nullptr;   // [i2][i0][i1] copy for the plane pass (n0 = n1 = 64 only)
  double* d_C64 = nullptr;
  float* d_C32 = nullptr;
  double* d_rho64 = nullptr;
  float* d_rho32 = nullptr;
  double* d_tw64[3] = {nullptr, nullptr, nullptr};
  float* d_tw32[3] = {nullptr, nullptr, nullptr};
  double* d_rhoinv64 = nullptr;  // 1 / rho' per grain
  float* d_rhoinv32 = nullptr;
  unsigned* d_ctr = nullptr;      // last-block counters (zero between launches)
  // workspaces
  bw::DevBuf ws_q, ws_q2, ws_pcg, ws_misc, ws_red, ws_red2;
  bw::Workspace<double> ws64;
  bw::Workspace<float> ws32;
  bw::Workspace<double> wl64;  // Lanczos bases
  bw::Workspace<float> wl32;
  bw::DevBuf ws_q3;
  double qcache_k[3] = {0, 0, 0};
  int qcache_nvec = -1;
  int pcg_counters_nvec = 0;
  // FFT schedule per axis (0, 1, 2): register kernels where the length allows
  // (tune_reg) and the cap on lines per tile of the generic LDS kernels (0 =
  // as many as fit); set by bw_autotune
  // [0]: FP32 kernels, [1]: FP64 kernels (a BW_MIXED cell runs both: the PCG in
  // FP32, the Rayleigh-Ritz refinement in FP64)
  int tune_reg[2][3] = {{1, 1, 1}, {1, 1, 1}};
  int tune_cap[2][3] = {{0, 0, 0}, {0, 0, 0}};
  int tune_plane = 1;   // FP32 cells with n0 = n1 = 64: the fused plane pass
  int tune_slab = 1;    // FP32 cells with n1 = n2 = 128: the three-pass slab path
  // cell groups (several cells of one grid in one batch; bw_lowest_modes_batched):
  // ncell cells, grain map [ncell][nvox], grain tables of all cells in one scale,
  // per-cell scaled C0 and smallest scaled density; csel maps the vectors of the
  // current launches to cells, kcell_bounds the wave vectors of the batched call
  int ncell = 1;
  bw::CellSel csel;
  std::vector<double> cell_C0s;      // ncell x 21
  std::vector<double> cell_rho_min;  // ncell
  std::vector<long> kcell_bounds;    // ncell + 1 (first wave vector of each cell)
  float* d_C0tab32 = nullptr;
  double* d_C0tab64 = nullptr;
  uint64_t serial = 0;               // unique per handle (group cache key)
  bw_rve* group = nullptr;           // cached group of this cell with others
  std::vector<uint64_t> group_key;
  // handles that share this cell's device tables but own their workspaces (the
  // concurrent wave-vector groups of one call); shared_tables marks such a clone
  std::vector<bw_rve*> clones;
  bool shared_tables = false;
  // captured PCG chunk (replayed with hipGraphLaunch while its key matches)
  hipStream_t cap_stream = nullptr;
  hipGraph_t pcg_graph = nullptr;
  hipGraphExec_t pcg_exec = nullptr;
  std::vector<const void*> pcg_key;
};

namespace bw {

// The group handle of nc >= 2 cells of one grid, cell edge and precision
// (created on first use and cached in cells[0]; freed with it).
bw_rve* cell_group(bw_rve* const* cells, int nc);
// Clone i (>= 1) of a cell for a concurrent wave-vector group: the cell's tables,
// scales and FFT schedule, workspaces of its own (created on first use, cached).
bw_rve* cell_clone(bw_rve* r, int i);

// q tables for a list of k (SI, rad/m); fills null_index.
QTable make_qtable(const bw_rve* r, const double* k_host, int nk);

// Launchers (defined per precision in bw_ops_impl.h).  All pointers are device
// pointers; qtab is a device table for nvec vectors.
template <typename T>
void launch_apply_K(const bw_rve* r, const double* d_qtab, const cplx<T>* u, cplx<T>* y, int nvec,
                    double scale, cplx<T>* W, hipStream_t s);
template <typename T>
void launch_apply_M(const bw_rve* r, const cplx<T>* u, cplx<T>* y, int nvec, double scale,
                    cplx<T>* W, hipStream_t s);
// y = scale * M u, or scale * M^-1 u when `inverse` (Sec. 3.3 eq. def_invM)
template <typename T>
void launch_apply_Minv_or_M(const bw_rve* r, const cplx<T>* u, cplx<T>* y, int nvec, bool inverse, cplx<T>* W,
                            hipStream_t s);
template <typename T>
void launch_apply_P(const bw_rve* r, const double* d_qtab, const cplx<T>* u, cplx<T>* y, int nvec,
                    double scale, hipStream_t s);

// PCG building blocks (bw_ops_impl.h)
struct PcgDev {
  // per-vector scalars and control, device
  double* rz;       // <r, z>
  double* pAp;      // <p, K p>
  double* alpha;
  double* beta;
  double* rr;       // ||r||^2
  double* bb;       // ||b||^2 * tol^2 (threshold)
  int* active;      // 1 while iterating
  int* iters;       // iterations per vector
  int* mask;        // restart selection
  double* partial;  // [nvec][max_blocks] partial sums (2 per block)
  unsigned* counter;  // [nvec] last-block counters
  int max_blocks;
  int maxit;        // a vector stops after this many iterations (with the convergence test)
};

// (on the FP32 slab path the update also leaves z = P^ r in Ap for the next direction)
template <typename T>
void launch_pcg_update(const bw_rve* r, const double* d_qtab, cplx<T>* x, cplx<T>* rv,
                       const cplx<T>* p, cplx<T>* Ap, int nvec, const PcgDev& pd,
                       hipStream_t s);
// ||r||^2 and ||b||^2 of a given residual (no writes)
template <typename T>
void launch_norms2(const bw_rve* r, const cplx<T>* b, const cplx<T>* rv, int nvec, double* d_rr, double* d_bb,
                   double* d_partial, int max_blocks, hipStream_t s);
// r = b - K x stored in rv (K x computed into tmp), with ||r||^2, ||b||^2 (FP64)
template <typename T>
void launch_residual(const bw_rve* r, const double* d_qtab, const cplx<T>* b, const cplx<T>* x,
                     cplx<T>* rv, cplx<T>* tmp, cplx<T>* W, int nvec, double* d_rr, double* d_bb,
                     double* d_partial, unsigned* d_counter, int max_blocks, hipStream_t s);
// z = P^ r, <r, z> -> rz, beta = 0 for restart (z also written to Ap on the FP32 slab path)
template <typename T>
void launch_pcg_restart(const bw_rve* r, const double* d_qtab, const cplx<T>* rv, int nvec,
                        const PcgDev& pd, const int* d_mask, hipStream_t s, cplx<T>* Ap);

template <typename T>
void launch_pcg_apply(const bw_rve* r, const double* d_qtab, const cplx<T>* rv, cplx<T>* p, cplx<T>* Ap,
                      cplx<T>* W, int nvec, const PcgDev& pd, hipStream_t s);
template <typename T> void scale_vectors(cplx<T>* x, size_t n, double sc, hipStream_t s);
template <typename T> void zero_voxel(cplx<T>* x, int nvec, long nvox, long vox, hipStream_t s);

// flexible PCG with the learned preconditioner on the scaled system K' x = b
// (bw_unet.hip); u null: the plain preconditioner
struct FpcgResult {
  std::vector<int> its, fb;    // iterations and fallbacks to the plain preconditioner, per right-hand side
  std::vector<double> rel;     // final true relative residuals
  long total = 0;
  bool conv = true;
};
FpcgResult fpcg_run(bw_rve* r, bw_unet* u, const double* dq, const QTable& qt, const float2* b, float2* x, int nrhs,
                    double rtol, int maxit, hipStream_t s);
// solver layer (bw_api.hip)
template <typename T> Workspace<T>& ws(bw_rve* r);
template <> inline Workspace<double>& ws<double>(bw_rve* r) { return r->ws64; }
template <> inline Workspace<float>& ws<float>(bw_rve* r) { return r->ws32; }
template <typename T> Workspace<T>& wl(bw_rve* r);
template <> inline Workspace<double>& wl<double>(bw_rve* r) { return r->wl64; }
template <> inline Workspace<float>& wl<float>(bw_rve* r) { return r->wl32; }
PcgDev pcg_dev(bw_rve* r, int nvec);
const double* upload_qtable(bw_rve* r, const QTable& t, DevBuf& buf, hipStream_t s);
double K_scale(const bw_rve* r);
double M_scale(const bw_rve* r);
// x0_zero: x is ignored, taken as 0 and first set to 0.  r_ready: the caller already wrote the
// initial residual b - K x into workspace vector 0.  true_check: confirm the
// recurrence residual with a true residual before returning.
template <typename T>
PcgResult pcg_run(bw_rve* r, const double* d_qtab, const QTable& qt, const cplx<T>* b, cplx<T>* x, int nvec,
                  double tol, int maxit, bool x0_zero, hipStream_t s, bool r_ready = false, bool true_check = true);

}  // namespace bw
