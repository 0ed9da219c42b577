// C-ABI entry points: cell creation, operator applies and the batched PCG
// solver (Sec. 3.3, Algorithm "InvA").
#include <chrono>
#include <cmath>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <cstring>

#include "bw_ops_impl.h"

namespace bw {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// ---------------------------------------------------------------------------
// kernel timing registry
// ---------------------------------------------------------------------------
namespace {
struct Pending {
  const char* name;
  hipEvent_t e0, e1;
  long units;
};
struct Totals {
  long launches = 0, units = 0;
  double ms = 0;
  std::vector<std::pair<float, float>> spans;   // launch intervals from g_ref (ms)
};
std::mutex g_tmu;
std::atomic<bool> g_timing{false};
std::string g_filter;  // time only this kernel name when non-empty
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, Totals> g_tot;
hipEvent_t g_ref = nullptr;   // recorded when timing is switched on

// total time during which at least one launch of a kernel ran (launches of one
// kernel on concurrent streams overlap; their summed durations would count the
// shared time more than once)
double union_ms(std::vector<std::pair<float, float>> v) {
  std::sort(v.begin(), v.end());
  double tot = 0, a = 0, b = -1;
  for (auto& x : v) {
    if (x.first > b) {
      if (b > a) tot += b - a;
      a = x.first;
      b = x.second;
    } else if (x.second > b) {
      b = x.second;
    }
  }
  if (b > a) tot += b - a;
  return tot;
}

hipEvent_t pool_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
void drain_locked() {
  for (auto& p : g_pending) {
    float ms = 0;
    if (p.e0 && p.e1 && hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      Totals& t = g_tot[p.name];
      t.launches += 1;
      t.ms += ms;
      t.units += p.units;
      float a = 0;
      if (g_ref && hipEventElapsedTime(&a, g_ref, p.e0) == hipSuccess) t.spans.push_back({a, a + ms});
    }
    if (p.e0) g_pool.push_back(p.e0);
    if (p.e1) g_pool.push_back(p.e1);
  }
  g_pending.clear();
}
}  // namespace

bool timing_enabled() { return g_timing.load(std::memory_order_relaxed); }

namespace {
std::atomic<bool> g_graphs{true};
}
std::recursive_mutex& capture_alloc_mutex() {
  static std::recursive_mutex m;
  return m;
}

// graphs are replayed only while no kernel timing is requested (timing brackets
// every launch with events, which a replayed graph cannot do)
bool graphs_enabled() { return g_graphs.load(std::memory_order_relaxed) && !timing_enabled(); }

KTimer::KTimer(const char* n, hipStream_t st, long u) : name(n), s(st), units(u) {
  if (!timing_enabled()) return;
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_filter.empty() && g_filter != n) return;
  e0 = pool_get();
  if (e0) (void)hipEventRecord(e0, s);
}
KTimer::~KTimer() {
  if (!e0) return;
  std::lock_guard<std::mutex> lk(g_tmu);
  hipEvent_t e1 = pool_get();
  if (e1) (void)hipEventRecord(e1, s);
  g_pending.push_back(Pending{name, e0, e1, units});
  if (g_pending.size() > 4096) drain_locked();
}
void timing_add_units(const char* name, long units) {
  if (!timing_enabled()) return;
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_filter.empty() && g_filter != name) return;
  g_tot[name].units += units;
}

// ---------------------------------------------------------------------------
// discrete frequencies (Sec. 3.1 eq. "frequencies", Sec. 3.2)
// ---------------------------------------------------------------------------
// Label stored at DFT index j: the paper's window shifted by whole reciprocal
// vectors so that the reduced wave number lies in (-1/2, 1/2].
static int window_lo(int N, double kappa) {
  const int paper_lo = -(N / 2);
  const int g = (int)std::ceil(kappa - 0.5 - 1e-9);
  return paper_lo - g;
}

QTable make_qtable(const bw_rve* r, const double* k_host, int nk) {
  QTable t;
  const int n[3] = {r->g.n0, r->g.n1, r->g.n2};
  const int per = n[0] + n[1] + n[2];
  t.nvec = nk;
  t.host.resize((size_t)nk * per);
  t.null_index.assign(nk, -1);
  for (int v = 0; v < nk; ++v) {
    int zero_at[3] = {-1, -1, -1};
    double* dst = t.host.data() + (size_t)v * per;
    for (int a = 0; a < 3; ++a) {
      double k = k_host[3 * v + a];
      double kappa = k * r->L[a] / (2.0 * M_PI);
      // within 1e-9 of a whole reciprocal vector: take that vector exactly, so
      // that xi + k = 0 on one voxel (K singular) is recognized
      const double g = std::nearbyint(kappa);
      if (std::fabs(kappa - g) <= 1e-9) {
        kappa = g;
        k = 2.0 * M_PI * g / r->L[a];
      }
      const int lo = window_lo(n[a], kappa);
      for (int j = 0; j < n[a]; ++j) {
        int mm = (j - lo) % n[a];
        if (mm < 0) mm += n[a];
        const int m = lo + mm;
        const double q = 2.0 * M_PI * m / r->L[a] + k;  // SI, as xi + k
        *dst++ = q * r->ell;
        if (q == 0.0) zero_at[a] = j;
      }
    }
    if (zero_at[0] >= 0 && zero_at[1] >= 0 && zero_at[2] >= 0)
      t.null_index[v] = (zero_at[0] * n[1] + zero_at[1]) * n[2] + zero_at[2];
  }
  return t;
}

// Upload a q table to `buf` through a pinned staging area.
const double* upload_qtable(bw_rve* r, const QTable& t, DevBuf& buf, hipStream_t s) {
  const size_t bytes = t.host.size() * sizeof(double);
  double* d = (double*)buf.get(bytes);
  h2d(d, t.host.data(), bytes, s);
  BW_HIP(hipStreamSynchronize(s));
  return d;
}

// Cached q table for a single k repeated nvec times (operator applies).
static const double* qtab_for(bw_rve* r, const double* k, int nvec, hipStream_t s) {
  if (r->qcache_nvec == nvec && std::memcmp(r->qcache_k, k, sizeof(r->qcache_k)) == 0 && r->ws_q.p)
    return (const double*)r->ws_q.p;
  std::vector<double> ks((size_t)nvec * 3);
  for (int v = 0; v < nvec; ++v)
    for (int a = 0; a < 3; ++a) ks[3 * v + a] = k[a];
  QTable t = make_qtable(r, ks.data(), nvec);
  const double* d = upload_qtable(r, t, r->ws_q, s);
  std::memcpy(r->qcache_k, k, sizeof(r->qcache_k));
  r->qcache_nvec = nvec;
  return d;
}

double K_scale(const bw_rve* r) { return r->Cref / (r->ell * r->ell); }
double M_scale(const bw_rve* r) { return r->rho_bar; }

// ---------------------------------------------------------------------------
// batched PCG on the scaled operator K' (Sec. 3.3, Algorithm "InvA")
// ---------------------------------------------------------------------------
template <typename T>
PcgResult pcg_run(bw_rve* r, const double* d_qtab, const QTable& qt, const cplx<T>* b, cplx<T>* x, int nvec,
                  double tol, int maxit, bool x0_zero, hipStream_t s, bool r_ready, bool true_check) {
  const Geom& g = r->g;
  const size_t n3 = (size_t)g.nvox * 3;
  PcgResult res;
  res.iters.assign(nvec, 0);
  res.relres.assign(nvec, 0.0);
  Workspace<T>& w = ws<T>(r);
  cplx<T>* rv = w.vec(0, (size_t)nvec * n3);
  cplx<T>* p = w.vec(1, (size_t)nvec * n3);
  cplx<T>* Ap = w.vec(2, (size_t)nvec * n3);
  cplx<T>* W = w.work((size_t)nvec * 6 * g.nvox);
  PcgDev pd = pcg_dev(r, nvec);
  pd.maxit = maxit;

  // x taken as 0: written as 0, so that a right-hand side that never iterates
  // (already converged, e.g. b = 0) returns 0 and the true-residual check sees it
  if (x0_zero) BW_HIP(hipMemsetAsync(x, 0, (size_t)nvec * n3 * sizeof(cplx<T>), s));
  if (r_ready) {
    launch_norms2<T>(r, b, rv, nvec, pd.rr, pd.rz /* ||b||^2 */, pd.partial, pd.max_blocks, s);
  } else {
    launch_residual<T>(r, d_qtab, b, x0_zero ? nullptr : x, rv, Ap, W, nvec, pd.rr, pd.rz /* ||b||^2 */,
                       pd.partial, pd.counter, pd.max_blocks, s);
    if (!x0_zero) res.k_applies += nvec;
  }
  std::vector<double> rr(nvec), bb(nvec), thr(nvec);
  BW_HIP(hipMemcpyAsync(rr.data(), pd.rr, nvec * sizeof(double), hipMemcpyDeviceToHost, s));
  BW_HIP(hipMemcpyAsync(bb.data(), pd.rz, nvec * sizeof(double), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  std::vector<int> act(nvec), it0(nvec, 0);
  bool zeroed = false;
  for (int v = 0; v < nvec; ++v) {
    thr[v] = tol * tol * bb[v];
    act[v] = rr[v] > thr[v] ? 1 : 0;
    if (bb[v] == 0 && act[v]) {
      // b = 0 with a nonzero start: the solution is 0 (no relative tolerance applies)
      BW_HIP(hipMemsetAsync(x + (size_t)v * n3, 0, n3 * sizeof(cplx<T>), s));
      rr[v] = 0;
      act[v] = 0;
      zeroed = true;
    }
  }
  if (zeroed) h2d(pd.rr, rr.data(), nvec * sizeof(double), s);
  h2d(pd.bb, thr.data(), nvec * sizeof(double), s);
  h2d(pd.active, act.data(), nvec * sizeof(int), s);
  h2d(pd.mask, act.data(), nvec * sizeof(int), s);
  h2d(pd.iters, it0.data(), nvec * sizeof(int), s);
  launch_pcg_restart<T>(r, d_qtab, rv, nvec, pd, pd.mask, s, Ap);
  BW_HIP(hipStreamSynchronize(s));

  // iterations per host check: a vector stops on the device when it converges or
  // reaches maxit, so the chunk length only sets how often the host looks
  const int chunk = 8;
  std::vector<int> its(nvec), mask(nvec, 0), its_prev(nvec, 0);
  int restarts = 0;
  for (;;) {
    bool any = false;
    for (int v = 0; v < nvec; ++v) any |= act[v] != 0;
    if (any) {
      if (graphs_enabled()) {
        // one chunk of iterations as a captured graph: identical launches with
        // identical arguments every time (per-vector scalars live on the device)
        std::vector<const void*> key = {(const void*)d_qtab, x, rv, p, Ap, W, pd.rz, pd.partial,
                                        (const void*)(long)nvec, (const void*)(long)chunk,
                                        (const void*)(long)sizeof(T), (const void*)(long)maxit,
                                        (const void*)(long)r->csel.n};
        // the cell selection is a kernel argument of the captured launches
        for (int i = 0; i + 1 < r->csel.n; ++i) key.push_back((const void*)(long)r->csel.bound[i]);
        if (!r->pcg_exec || r->pcg_key != key) {
          // no allocation or free on another thread while this thread captures
          std::lock_guard<std::recursive_mutex> lk(capture_alloc_mutex());
          if (r->pcg_exec) (void)hipGraphExecDestroy(r->pcg_exec);
          if (r->pcg_graph) (void)hipGraphDestroy(r->pcg_graph);
          r->pcg_exec = nullptr;
          r->pcg_graph = nullptr;
          r->pcg_key.clear();
          if (!r->cap_stream) BW_HIP(hipStreamCreateWithFlags(&r->cap_stream, hipStreamNonBlocking));
          BW_HIP(hipStreamSynchronize(s));
          BW_HIP(hipStreamBeginCapture(r->cap_stream, hipStreamCaptureModeThreadLocal));
          for (int c = 0; c < chunk; ++c) {
            launch_pcg_apply<T>(r, d_qtab, rv, p, Ap, W, nvec, pd, r->cap_stream);
            launch_pcg_update<T>(r, d_qtab, x, rv, p, Ap, nvec, pd, r->cap_stream);
          }
          hipGraph_t gr = nullptr;
          BW_HIP(hipStreamEndCapture(r->cap_stream, &gr));
          r->pcg_graph = gr;
          BW_HIP(hipGraphInstantiate(&r->pcg_exec, gr, nullptr, nullptr, 0));
          r->pcg_key = key;
        }
        BW_HIP(hipGraphLaunch(r->pcg_exec, s));
        res.block_iters += chunk;
      } else {
        for (int c = 0; c < chunk; ++c) {
          launch_pcg_apply<T>(r, d_qtab, rv, p, Ap, W, nvec, pd, s);
          launch_pcg_update<T>(r, d_qtab, x, rv, p, Ap, nvec, pd, s);
          res.block_iters += 1;
        }
      }
      BW_HIP(hipMemcpyAsync(act.data(), pd.active, nvec * sizeof(int), hipMemcpyDeviceToHost, s));
      BW_HIP(hipMemcpyAsync(its.data(), pd.iters, nvec * sizeof(int), hipMemcpyDeviceToHost, s));
      BW_HIP(hipStreamSynchronize(s));
      if (timing_enabled()) {
        long d = 0;
        for (int v = 0; v < nvec; ++v) d += its[v] - its_prev[v];
        its_prev = its;
        for (const char* nm : {"k_strain_row_pcg", "k_axis1_inv_pcg", "k_axis0_contract_pcg", "k_axis1_fwd_pcg",
                               "k_plane_contract_pcg", "k_row_div_pcg", "k_slab_strain_pcg", "k_slab_div_pcg",
                               "k_pcg_update", "k_pcg_update_z"})
          timing_add_units(nm, d);
      }
      bool cap = false;
      for (int v = 0; v < nvec; ++v)
        if (act[v] && its[v] >= maxit) {
          act[v] = 0;
          cap = true;
        }
      if (cap) h2d(pd.active, act.data(), nvec * sizeof(int), s);
      any = false;
      for (int v = 0; v < nvec; ++v) any |= act[v] != 0;
      if (any) continue;
    }
    // every vector stopped: check the true residual (or take the recurrence's)
    if (true_check) {
      launch_residual<T>(r, d_qtab, b, x, rv, Ap, W, nvec, pd.rr, nullptr, pd.partial, pd.counter, pd.max_blocks,
                         s);
      res.k_applies += nvec;
    }
    BW_HIP(hipMemcpyAsync(rr.data(), pd.rr, nvec * sizeof(double), hipMemcpyDeviceToHost, s));
    BW_HIP(hipMemcpyAsync(its.data(), pd.iters, nvec * sizeof(int), hipMemcpyDeviceToHost, s));
    BW_HIP(hipStreamSynchronize(s));
    bool again = false;
    std::fill(mask.begin(), mask.end(), 0);
    for (int v = 0; v < nvec && true_check; ++v) {
      if (rr[v] > thr[v] && its[v] < maxit && restarts < 8) {
        mask[v] = 1;
        again = true;
      }
    }
    if (!again) break;
    ++restarts;
    act = mask;
    h2d(pd.active, act.data(), nvec * sizeof(int), s);
    h2d(pd.mask, mask.data(), nvec * sizeof(int), s);
    launch_pcg_restart<T>(r, d_qtab, rv, nvec, pd, pd.mask, s, Ap);
  }
  res.converged = true;
  for (int v = 0; v < nvec; ++v) {
    res.iters[v] = its[v];
    res.relres[v] = bb[v] > 0 ? std::sqrt(rr[v] / bb[v]) : 0.0;
    if (rr[v] > thr[v]) res.converged = false;
    res.total_iters += its[v];
  }
  res.k_applies += res.total_iters;
  return res;
}

template PcgResult pcg_run<double>(bw_rve*, const double*, const QTable&, const cplx<double>*, cplx<double>*, int,
                                   double, int, bool, hipStream_t, bool, bool);
template PcgResult pcg_run<float>(bw_rve*, const double*, const QTable&, const cplx<float>*, cplx<float>*, int,
                                  double, int, bool, hipStream_t, bool, bool);

PcgDev pcg_dev(bw_rve* r, int nvec) {
  const Geom& g = r->g;
  // blocks per vector of every reducing kernel: row tiles (<= n0 n1) and the
  // pointwise kernels
  int maxb = std::max(pw_blocks(g.nvox * 3), (int)std::max<long>(1, (long)g.n0 * g.n1));
  const size_t dbl = (size_t)nvec * 8;
  const size_t part = (size_t)nvec * maxb * 2;
  const size_t ints = (size_t)nvec * 4;
  char* base = (char*)r->ws_pcg.get((dbl + part) * sizeof(double) + ints * sizeof(int) + 256);
  PcgDev pd{};
  double* d = (double*)base;
  pd.rz = d;
  pd.pAp = d + nvec;
  pd.alpha = d + 2 * nvec;
  pd.beta = d + 3 * nvec;
  pd.rr = d + 4 * nvec;
  pd.bb = d + 5 * nvec;
  pd.partial = d + dbl;
  int* ip = (int*)(d + dbl + part);
  pd.active = ip;
  pd.iters = ip + nvec;
  pd.mask = ip + 2 * nvec;
  pd.counter = (unsigned*)(ip + 3 * nvec);
  pd.max_blocks = maxb;
  pd.maxit = 0x7fffffff;
  if (r->pcg_counters_nvec < nvec) {
    BW_HIP(hipMemset(pd.counter, 0, nvec * sizeof(unsigned)));
    r->pcg_counters_nvec = nvec;
  }
  return pd;
}

// ---------------------------------------------------------------------------
// workspaces
// ---------------------------------------------------------------------------

}  // namespace bw

using namespace bw;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define BW_GUARD_BEGIN try {
#define BW_GUARD_END                               \
  }                                                \
  catch (const bw::Error& e) {                     \
    bw::set_error(e.msg);                          \
    return e.code;                                 \
  }                                                \
  catch (const std::exception& e) {                \
    bw::set_error(std::string("internal: ") + e.what()); \
    return BW_EINVAL;                              \
  }

extern "C" const char* bw_last_error(void) { return g_last_error.c_str(); }

extern "C" int bw_timing_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_tmu);
  drain_locked();
  g_tot.clear();
  if (enable) {
    if (!g_ref && hipEventCreate(&g_ref) != hipSuccess) g_ref = nullptr;
    if (g_ref) (void)hipEventRecord(g_ref, nullptr);
  }
  g_timing.store(enable != 0);
  return BW_OK;
}

extern "C" int bw_graphs_enable(int32_t enable) {
  g_graphs.store(enable != 0);
  return BW_OK;
}

extern "C" int bw_timing_filter(const char* kernel_name) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_filter = kernel_name ? kernel_name : "";
  return BW_OK;
}

namespace bw {
// plain streaming copy (16-byte words, one per thread over a full grid: the
// resident workgroups then stream neighbouring memory, measured faster than a
// grid-stride loop), the calibration kernel for memory counters and the
// device-copy bandwidth reference
__global__ void k_diag_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[e];
}
}  // namespace bw

extern "C" int bw_diag_copy(const void* src, void* dst, int64_t bytes, void* stream) {
  BW_GUARD_BEGIN
  BW_REQUIRE(src && dst, BW_EINVAL, "null argument");
  BW_REQUIRE(bytes >= 0 && bytes % 16 == 0, BW_EINVAL, "bytes must be a non-negative multiple of 16");
  BW_REQUIRE(((uintptr_t)src | (uintptr_t)dst) % 16 == 0, BW_EINVAL, "buffers must be 16-byte aligned");
  const long n = bytes / 16;
  if (n == 0) return BW_OK;
  const long blocks = (n + 255) / 256;
  BW_REQUIRE(blocks < (1L << 31), BW_EINVAL, "copy too large");
  BW_LAUNCH("k_diag_copy", 0, k_diag_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
            (const uint4*)src, (uint4*)dst, n);
  BW_HIP(hipGetLastError());
  return BW_OK;
  BW_GUARD_END
}

extern "C" int64_t bw_timing_report(char* buf, int64_t len) {
  std::lock_guard<std::mutex> lk(g_tmu);
  drain_locked();
  std::string js = "{";
  bool first = true;
  for (auto& kv : g_tot) {
    char tmp[256];
    snprintf(tmp, sizeof(tmp), "%s\"%s\": {\"launches\": %ld, \"ms\": %.6f, \"units\": %ld, \"union_ms\": %.6f}",
             first ? "" : ", ", kv.first.c_str(), kv.second.launches, kv.second.ms, kv.second.units,
             kv.second.spans.size() == (size_t)kv.second.launches ? union_ms(kv.second.spans) : kv.second.ms);
    js += tmp;
    first = false;
  }
  js += "}";
  if (buf && len > 0) {
    const size_t n = std::min<size_t>(js.size(), (size_t)len - 1);
    std::memcpy(buf, js.data(), n);
    buf[n] = 0;
  }
  return (int64_t)js.size() + 1;
}

static bool spd6(const double* c21) {
  // Cholesky of the symmetric 6x6
  double A[6][6];
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) A[a][b] = c21[vidx(a, b)];
  for (int j = 0; j < 6; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    A[j][j] = d;
    for (int i = j + 1; i < 6; ++i) {
      double v = A[i][j];
      for (int k = 0; k < j; ++k) v -= A[i][k] * A[j][k];
      A[i][j] = v / d;
    }
  }
  return true;
}

// Device copies of a cell's (or a cell group's) tables: grain map(s) (ncell x
// nvox; the transposed copy for the plane pass at n0 = n1 = 64), scaled stiffness
// and density tables of all grains, inverse densities, counters, twiddles, and
// for a group the per-cell reference stiffness rows.
static void upload_cell_tables(bw_rve* r, const uint16_t* grain_map_host) {
  const int n[3] = {r->g.n0, r->g.n1, r->g.n2};
  const long nvox = r->g.nvox;
  const long nmap = nvox * r->ncell;
  const int n_grains = r->G;
  std::vector<float> c32(r->C21s_host.begin(), r->C21s_host.end());
  std::vector<float> r32(r->rhos_host.begin(), r->rhos_host.end());
  std::vector<double> ri64(n_grains);
  std::vector<float> ri32(n_grains);
  for (int gi = 0; gi < n_grains; ++gi) {
    ri64[gi] = 1.0 / r->rhos_host[gi];
    ri32[gi] = (float)ri64[gi];
  }
  BW_HIP(hipMalloc(&r->d_rhoinv64, n_grains * sizeof(double)));
  BW_HIP(hipMalloc(&r->d_rhoinv32, n_grains * sizeof(float)));
  BW_HIP(hipMemcpy(r->d_rhoinv64, ri64.data(), n_grains * sizeof(double), hipMemcpyHostToDevice));
  BW_HIP(hipMemcpy(r->d_rhoinv32, ri32.data(), n_grains * sizeof(float), hipMemcpyHostToDevice));
  BW_HIP(hipMalloc(&r->d_ctr, 1024 * sizeof(unsigned)));
  BW_HIP(hipMemset(r->d_ctr, 0, 1024 * sizeof(unsigned)));
  BW_HIP(hipMalloc(&r->d_gmap, nmap * sizeof(uint16_t)));
  BW_HIP(hipMalloc(&r->d_C64, r->C21s_host.size() * sizeof(double)));
  BW_HIP(hipMalloc(&r->d_C32, c32.size() * sizeof(float)));
  BW_HIP(hipMalloc(&r->d_rho64, n_grains * sizeof(double)));
  BW_HIP(hipMalloc(&r->d_rho32, n_grains * sizeof(float)));
  BW_HIP(hipMemcpy(r->d_gmap, grain_map_host, nmap * sizeof(uint16_t), hipMemcpyHostToDevice));
  if (n[0] == 64 && n[1] == 64) {
    std::vector<uint16_t> gt(nmap);
    for (long c = 0; c < r->ncell; ++c)
      for (long i0 = 0; i0 < 64; ++i0)
        for (long i1 = 0; i1 < 64; ++i1)
          for (long i2 = 0; i2 < n[2]; ++i2)
            gt[c * nvox + (i2 * 64 + i0) * 64 + i1] = grain_map_host[c * nvox + (i0 * 64 + i1) * n[2] + i2];
    BW_HIP(hipMalloc(&r->d_gmapT, nmap * sizeof(uint16_t)));
    BW_HIP(hipMemcpy(r->d_gmapT, gt.data(), nmap * sizeof(uint16_t), hipMemcpyHostToDevice));
  }
  BW_HIP(hipMemcpy(r->d_C64, r->C21s_host.data(), r->C21s_host.size() * sizeof(double), hipMemcpyHostToDevice));
  BW_HIP(hipMemcpy(r->d_C32, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice));
  BW_HIP(hipMemcpy(r->d_rho64, r->rhos_host.data(), n_grains * sizeof(double), hipMemcpyHostToDevice));
  BW_HIP(hipMemcpy(r->d_rho32, r32.data(), n_grains * sizeof(float), hipMemcpyHostToDevice));
  // twiddle tables exp(-2 pi i t / N), computed in long double
  for (int a = 0; a < 3; ++a) {
    const int N = n[a];
    std::vector<double> t64(2 * N);
    std::vector<float> t32(2 * N);
    for (int t = 0; t < N; ++t) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)N;
      t64[2 * t] = (double)cosl(ang);
      t64[2 * t + 1] = (double)sinl(ang);
      t32[2 * t] = (float)cosl(ang);
      t32[2 * t + 1] = (float)sinl(ang);
    }
    BW_HIP(hipMalloc(&r->d_tw64[a], 2 * N * sizeof(double)));
    BW_HIP(hipMalloc(&r->d_tw32[a], 2 * N * sizeof(float)));
    BW_HIP(hipMemcpy(r->d_tw64[a], t64.data(), 2 * N * sizeof(double), hipMemcpyHostToDevice));
    BW_HIP(hipMemcpy(r->d_tw32[a], t32.data(), 2 * N * sizeof(float), hipMemcpyHostToDevice));
  }
  if (r->ncell > 1) {
    std::vector<float> t32(r->cell_C0s.begin(), r->cell_C0s.end());
    BW_HIP(hipMalloc(&r->d_C0tab64, r->cell_C0s.size() * sizeof(double)));
    BW_HIP(hipMalloc(&r->d_C0tab32, t32.size() * sizeof(float)));
    BW_HIP(hipMemcpy(r->d_C0tab64, r->cell_C0s.data(), r->cell_C0s.size() * sizeof(double), hipMemcpyHostToDevice));
    BW_HIP(hipMemcpy(r->d_C0tab32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
  }
}

static uint64_t next_serial() {
  static std::atomic<uint64_t> ctr{0};
  return ++ctr;
}

extern "C" int bw_create_rve(bw_rve** out, const int32_t n[3], const double L[3], const uint16_t* grain_map_host,
                             int32_t n_grains, const double* C21_host, const double* rho_host, int32_t precision,
                             void* stream) {
  BW_GUARD_BEGIN
  BW_REQUIRE(out && n && L && grain_map_host && C21_host && rho_host, BW_EINVAL, "null argument");
  *out = nullptr;
  BW_REQUIRE(precision == BW_FP64 || precision == BW_MIXED, BW_EINVAL, "precision must be BW_FP64 or BW_MIXED");
  BW_REQUIRE(n_grains >= 1 && n_grains <= 65535, BW_EINVAL, "n_grains out of range");
  for (int a = 0; a < 3; ++a) {
    BW_REQUIRE(n[a] >= 1, BW_EINVAL, "grid size must be >= 1");
    BW_REQUIRE(L[a] > 0 && std::isfinite(L[a]), BW_EINVAL, "cell edge must be > 0");
    BW_REQUIRE(size_supported(n[a]), BW_EUNSUPPORTED, "no compiled FFT of length " + std::to_string(n[a]));
  }
  const long nvox = (long)n[0] * n[1] * n[2];
  BW_REQUIRE(nvox <= (1L << 30), BW_EINVAL, "grid too large");
  for (int gi = 0; gi < n_grains; ++gi) {
    BW_REQUIRE(rho_host[gi] > 0 && std::isfinite(rho_host[gi]), BW_EINVAL, "density must be > 0");
    for (int i = 0; i < 21; ++i) BW_REQUIRE(std::isfinite(C21_host[gi * 21 + i]), BW_EINVAL, "non-finite stiffness");
    BW_REQUIRE(spd6(C21_host + gi * 21), BW_EINVAL,
               "stiffness of grain " + std::to_string(gi) + " is not positive definite");
  }
  std::vector<long> count(n_grains, 0);
  for (long i = 0; i < nvox; ++i) {
    BW_REQUIRE(grain_map_host[i] < n_grains, BW_EINVAL, "grain index out of range");
    count[grain_map_host[i]]++;
  }
  hipStream_t s = (hipStream_t)stream;
  auto* r = new bw_rve();
  try {
    r->g = Geom{n[0], n[1], n[2], nvox};
    for (int a = 0; a < 3; ++a) r->L[a] = L[a];
    r->G = n_grains;
    r->precision = precision;
    BW_HIP(hipGetDevice(&r->device));
    BW_HIP(hipDeviceGetAttribute(&r->ncu, hipDeviceAttributeMultiprocessorCount, r->device));
    // volume averages (Sec. 3.3: C0 = volume-averaged stiffness)
    double rs = 0;
    for (int i = 0; i < 21; ++i) r->C0_si[i] = 0;
    for (int gi = 0; gi < n_grains; ++gi) {
      const double w = (double)count[gi] / (double)nvox;
      for (int i = 0; i < 21; ++i) r->C0_si[i] += w * C21_host[gi * 21 + i];
      rs += w * rho_host[gi];
    }
    r->rho_bar = rs;
    {
      // one density in every occupied grain: take it as the mean exactly, so that the
      // scaled density is exactly 1 and M' is the identity (the solvers then copy
      // instead of transforming, and the Lanczos basis is its own M-image)
      double r0 = -1;
      bool uni = true;
      for (int gi = 0; gi < n_grains && uni; ++gi) {
        if (count[gi] == 0) continue;
        if (r0 < 0) r0 = rho_host[gi];
        else if (rho_host[gi] != r0) uni = false;
      }
      if (uni && r0 > 0) {
        r->rho_bar = r0;
        r->rho_unit = 1;
      }
    }
    r->Cref = r->C0_si[0];
    r->ell = L[0] / (2.0 * M_PI);
    for (int i = 0; i < 21; ++i) r->C0s[i] = r->C0_si[i] / r->Cref;
    r->C21s_host.resize((size_t)n_grains * 21);
    r->rhos_host.resize(n_grains);
    r->rho_min_s = INFINITY;
    for (int gi = 0; gi < n_grains; ++gi) {
      for (int i = 0; i < 21; ++i) r->C21s_host[gi * 21 + i] = C21_host[gi * 21 + i] / r->Cref;
      r->rhos_host[gi] = rho_host[gi] / r->rho_bar;
      if (count[gi] > 0) r->rho_min_s = std::min(r->rho_min_s, r->rhos_host[gi]);
    }
    upload_cell_tables(r, grain_map_host);
    r->serial = next_serial();
    (void)s;
  } catch (...) {
    bw_destroy_rve(r);
    throw;
  }
  *out = r;
  return BW_OK;
  BW_GUARD_END
}

namespace bw {

// A cell group: nc cells of one grid, cell edge and precision as one handle whose
// vectors carry their cell (CellSel).  Grain maps are stacked with the grain
// indices of cell c offset by the grains of the cells before it; all tables
// share the first cell's scales (C' = C / Cref, rho' = rho / rho_bar), so K, M and
// their eigenvalues keep one unit; every cell keeps its own reference stiffness C0
// (the preconditioner) and smallest density (the bounds).  Cached in the first
// cell's handle while the same cells are grouped again.
bw_rve* cell_group(bw_rve* const* cells, int nc) {
  BW_REQUIRE(nc >= 2 && nc <= CELLS_MAX, BW_EINVAL, "cell group size out of range");
  bw_rve* c0 = cells[0];
  std::vector<uint64_t> key(nc);
  for (int c = 0; c < nc; ++c) key[c] = cells[c]->serial;
  if (c0->group && c0->group_key == key) return c0->group;
  if (c0->group) {
    bw_destroy_rve(c0->group);
    c0->group = nullptr;
    c0->group_key.clear();
  }
  const long nvox = c0->g.nvox;
  int G = 0;
  for (int c = 0; c < nc; ++c) {
    const bw_rve* x = cells[c];
    BW_REQUIRE(x->ncell == 1, BW_EINVAL, "a cell group cannot contain a group");
    BW_REQUIRE(x->g.n0 == c0->g.n0 && x->g.n1 == c0->g.n1 && x->g.n2 == c0->g.n2 && x->precision == c0->precision &&
                   x->device == c0->device && x->L[0] == c0->L[0] && x->L[1] == c0->L[1] && x->L[2] == c0->L[2],
               BW_EINVAL, "cells of a group need one grid, cell edge, precision and device");
    G += x->G;
  }
  BW_REQUIRE(G <= 65535, BW_EINVAL, "too many grains in a cell group");
  std::vector<uint16_t> gm((size_t)nc * nvox);
  auto* r = new bw_rve();
  try {
    r->g = c0->g;
    for (int a = 0; a < 3; ++a) r->L[a] = c0->L[a];
    r->G = G;
    r->precision = c0->precision;
    r->device = c0->device;
    r->ncu = c0->ncu;
    r->Cref = c0->Cref;
    r->ell = c0->ell;
    r->rho_bar = c0->rho_bar;
    for (int i = 0; i < 21; ++i) {
      r->C0_si[i] = c0->C0_si[i];
      r->C0s[i] = c0->C0s[i];
    }
    r->ncell = nc;
    r->rho_unit = 1;
    r->rho_min_s = INFINITY;
    r->C21s_host.reserve((size_t)G * 21);
    r->rhos_host.reserve(G);
    int goff = 0;
    for (int c = 0; c < nc; ++c) {
      const bw_rve* x = cells[c];
      BW_HIP(hipMemcpy(gm.data() + (size_t)c * nvox, x->d_gmap, nvox * sizeof(uint16_t), hipMemcpyDeviceToHost));
      for (long i = 0; i < nvox; ++i) gm[(size_t)c * nvox + i] = (uint16_t)(gm[(size_t)c * nvox + i] + goff);
      const double cs = x->Cref / r->Cref, rs = x->rho_bar / r->rho_bar;
      for (int gi = 0; gi < x->G; ++gi) {
        for (int i = 0; i < 21; ++i) r->C21s_host.push_back(x->C21s_host[(size_t)gi * 21 + i] * cs);
        r->rhos_host.push_back(x->rhos_host[gi] * rs);
      }
      for (int i = 0; i < 21; ++i) r->cell_C0s.push_back(x->C0_si[i] / r->Cref);
      r->cell_rho_min.push_back(x->rho_min_s * rs);
      r->rho_min_s = std::min(r->rho_min_s, x->rho_min_s * rs);
      if (!(x->rho_unit && x->rho_bar == r->rho_bar)) r->rho_unit = 0;
      goff += x->G;
    }
    for (int t = 0; t < 2; ++t)
      for (int a = 0; a < 3; ++a) {
        r->tune_reg[t][a] = c0->tune_reg[t][a];
        r->tune_cap[t][a] = c0->tune_cap[t][a];
      }
    r->tune_plane = c0->tune_plane;
    r->tune_slab = c0->tune_slab;
    upload_cell_tables(r, gm.data());
    r->serial = next_serial();
  } catch (...) {
    bw_destroy_rve(r);
    throw;
  }
  c0->group = r;
  c0->group_key = key;
  return r;
}

bw_rve* cell_clone(bw_rve* r, int i) {
  BW_REQUIRE(i >= 1 && r->ncell == 1 && !r->shared_tables, BW_EINVAL, "no clone of this handle");
  if ((int)r->clones.size() < i) r->clones.resize(i, nullptr);
  bw_rve*& c = r->clones[i - 1];
  if (!c) {
    auto* x = new bw_rve();
    try {
      x->shared_tables = true;
      x->g = r->g;
      for (int a = 0; a < 3; ++a) x->L[a] = r->L[a];
      x->G = r->G;
      x->precision = r->precision;
      x->device = r->device;
      x->ncu = r->ncu;
      x->Cref = r->Cref;
      x->ell = r->ell;
      x->rho_bar = r->rho_bar;
      x->rho_min_s = r->rho_min_s;
      x->rho_unit = r->rho_unit;
      for (int k = 0; k < 21; ++k) {
        x->C0_si[k] = r->C0_si[k];
        x->C0s[k] = r->C0s[k];
      }
      x->C21s_host = r->C21s_host;
      x->rhos_host = r->rhos_host;
      x->d_gmap = r->d_gmap;
      x->d_gmapT = r->d_gmapT;
      x->d_C64 = r->d_C64;
      x->d_C32 = r->d_C32;
      x->d_rho64 = r->d_rho64;
      x->d_rho32 = r->d_rho32;
      x->d_rhoinv64 = r->d_rhoinv64;
      x->d_rhoinv32 = r->d_rhoinv32;
      for (int a = 0; a < 3; ++a) {
        x->d_tw64[a] = r->d_tw64[a];
        x->d_tw32[a] = r->d_tw32[a];
      }
      BW_HIP(hipMalloc(&x->d_ctr, 1024 * sizeof(unsigned)));
      BW_HIP(hipMemset(x->d_ctr, 0, 1024 * sizeof(unsigned)));
      x->serial = next_serial();
    } catch (...) {
      bw_destroy_rve(x);
      throw;
    }
    c = x;
  }
  // the parent's current FFT schedule
  for (int t = 0; t < 2; ++t)
    for (int a = 0; a < 3; ++a) {
      c->tune_reg[t][a] = r->tune_reg[t][a];
      c->tune_cap[t][a] = r->tune_cap[t][a];
    }
  c->tune_plane = r->tune_plane;
  c->tune_slab = r->tune_slab;
  return c;
}

}  // namespace bw

extern "C" void bw_destroy_rve(bw_rve* r) {
  if (!r) return;
  if (r->pcg_exec) (void)hipGraphExecDestroy(r->pcg_exec);
  if (r->pcg_graph) (void)hipGraphDestroy(r->pcg_graph);
  if (r->cap_stream) (void)hipStreamDestroy(r->cap_stream);
  for (bw_rve* c : r->clones)
    if (c) bw_destroy_rve(c);
  if (!r->shared_tables) {   // a clone's tables belong to its parent
    (void)hipFree(r->d_gmap);
    (void)hipFree(r->d_gmapT);
    (void)hipFree(r->d_C64);
    (void)hipFree(r->d_C32);
    (void)hipFree(r->d_rho64);
    (void)hipFree(r->d_rho32);
    (void)hipFree(r->d_rhoinv64);
    (void)hipFree(r->d_rhoinv32);
    (void)hipFree(r->d_C0tab32);
    (void)hipFree(r->d_C0tab64);
    for (int a = 0; a < 3; ++a) {
      (void)hipFree(r->d_tw64[a]);
      (void)hipFree(r->d_tw32[a]);
    }
  }
  (void)hipFree(r->d_ctr);
  if (r->group) bw_destroy_rve(r->group);
  r->ws_q.release();
  r->ws_q2.release();
  r->ws_red.release();
  r->ws_red2.release();
  r->ws_pcg.release();
  r->ws_misc.release();
  r->ws64.release();
  r->ws32.release();
  r->wl64.release();
  r->wl32.release();
  r->ws_q3.release();
  delete r;
}

extern "C" int bw_rve_info(const bw_rve* r, int32_t n[3], int32_t* precision, double C0_21[21], double* rho_bar) {
  BW_GUARD_BEGIN
  BW_REQUIRE(r, BW_EINVAL, "null cell");
  if (n) {
    n[0] = r->g.n0;
    n[1] = r->g.n1;
    n[2] = r->g.n2;
  }
  if (precision) *precision = r->precision;
  if (C0_21)
    for (int i = 0; i < 21; ++i) C0_21[i] = r->C0_si[i];
  if (rho_bar) *rho_bar = r->rho_bar;
  return BW_OK;
  BW_GUARD_END
}

extern "C" int bw_apply_K(bw_rve* r, const double k[3], const void* u, void* y, int32_t nvec, void* stream) {
  BW_GUARD_BEGIN
  BW_REQUIRE(r && k, BW_EINVAL, "null argument");
  BW_REQUIRE(nvec >= 0, BW_EINVAL, "nvec < 0");
  if (nvec == 0) return BW_OK;
  BW_REQUIRE(u && y, BW_EINVAL, "null argument");
  BW_REQUIRE(u != y, BW_EINVAL, "u and y must not alias");
  hipStream_t s = (hipStream_t)stream;
  const double* q = qtab_for(r, k, nvec, s);
  if (r->precision == BW_FP64) {
    auto* W = ws<double>(r).work((size_t)nvec * 6 * r->g.nvox);
    launch_apply_K<double>(r, q, (const cplx<double>*)u, (cplx<double>*)y, nvec, K_scale(r), W, s);
  } else {
    auto* W = ws<float>(r).work((size_t)nvec * 6 * r->g.nvox);
    launch_apply_K<float>(r, q, (const cplx<float>*)u, (cplx<float>*)y, nvec, K_scale(r), W, s);
  }
  BW_HIP(hipGetLastError());
  return BW_OK;
  BW_GUARD_END
}

extern "C" int bw_apply_M(bw_rve* r, const void* u, void* y, int32_t nvec, void* stream) {
  BW_GUARD_BEGIN
  BW_REQUIRE(r, BW_EINVAL, "null argument");
  BW_REQUIRE(nvec >= 0, BW_EINVAL, "nvec < 0");
  if (nvec == 0) return BW_OK;
  BW_REQUIRE(u && y, BW_EINVAL, "null argument");
  BW_REQUIRE(u != y, BW_EINVAL, "u and y must not alias");
  hipStream_t s = (hipStream_t)stream;
  if (r->precision == BW_FP64) {
    auto* W = ws<double>(r).work((size_t)nvec * 6 * r->g.nvox);
    launch_apply_M<double>(r, (const cplx<double>*)u, (cplx<double>*)y, nvec, M_scale(r), W, s);
  } else {
    auto* W = ws<float>(r).work((size_t)nvec * 6 * r->g.nvox);
    launch_apply_M<float>(r, (const cplx<float>*)u, (cplx<float>*)y, nvec, M_scale(r), W, s);
  }
  BW_HIP(hipGetLastError());
  return BW_OK;
  BW_GUARD_END
}

extern "C" int bw_apply_P(bw_rve* r, const double k[3], const void* u, void* y, int32_t nvec, void* stream) {
  BW_GUARD_BEGIN
  BW_REQUIRE(r && k, BW_EINVAL, "null argument");
  BW_REQUIRE(nvec >= 0, BW_EINVAL, "nvec < 0");
  if (nvec == 0) return BW_OK;
  BW_REQUIRE(u && y, BW_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  const double* q = qtab_for(r, k, nvec, s);
  const double sc = 1.0 / K_scale(r);
  if (r->precision == BW_FP64)
    launch_apply_P<double>(r, q, (const cplx<double>*)u, (cplx<double>*)y, nvec, sc, s);
  else
    launch_apply_P<float>(r, q, (const cplx<float>*)u, (cplx<float>*)y, nvec, sc, s);
  BW_HIP(hipGetLastError());
  return BW_OK;
  BW_GUARD_END
}

// ---------------------------------------------------------------------------
// FFT schedule: register kernels on/off and tile caps per axis, chosen by timing
// ---------------------------------------------------------------------------
static void drop_graph(bw_rve* r) {
  if (r->pcg_exec) (void)hipGraphExecDestroy(r->pcg_exec);
  if (r->pcg_graph) (void)hipGraphDestroy(r->pcg_graph);
  r->pcg_exec = nullptr;
  r->pcg_graph = nullptr;
  r->pcg_key.clear();
}

template <typename T> static int generic_lines(const bw_rve* r, int axis) {
  const Geom& g = r->g;
  if (axis == 2) return row_tile<T>(g.n2, (long)g.n0 * g.n1).NR;
  if (axis == 1) return axis1_tile<T>(g.n1, g.n2, 6L * g.n0 * g.n2).LT;
  return axis0_tile<T>(g.n0, (long)g.n1 * g.n2).LT;
}

template <typename T> static double autotune_impl(bw_rve* r, int nvec, hipStream_t s) {
  const Geom& g = r->g;
  DevBuf ub, yb;
  cplx<T>* u = (cplx<T>*)ub.get((size_t)nvec * 3 * g.nvox * sizeof(cplx<T>));
  cplx<T>* y = (cplx<T>*)yb.get((size_t)nvec * 3 * g.nvox * sizeof(cplx<T>));
  BW_HIP(hipMemsetAsync(u, 0, (size_t)nvec * 3 * g.nvox * sizeof(cplx<T>), s));
  const double k[3] = {0.3 * M_PI / r->L[0], 0.1 * M_PI / r->L[1], 0.05 * M_PI / r->L[2]};
  const double* q = qtab_for(r, k, nvec, s);
  cplx<T>* W = ws<T>(r).work((size_t)nvec * 6 * g.nvox);
  hipEvent_t e0, e1;
  BW_HIP(hipEventCreate(&e0));
  BW_HIP(hipEventCreate(&e1));
  auto time_apply = [&]() {
    launch_apply_K<T>(r, q, u, y, nvec, 1.0, W, s);
    BW_HIP(hipEventRecord(e0, s));
    for (int rep = 0; rep < 3; ++rep) launch_apply_K<T>(r, q, u, y, nvec, 1.0, W, s);
    BW_HIP(hipEventRecord(e1, s));
    BW_HIP(hipEventSynchronize(e1));
    float ms = 0;
    BW_HIP(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms / 3.0;
  };
  constexpr int ts = tsel<T>;
  for (int a = 0; a < 3; ++a) {
    r->tune_reg[ts][a] = 1;
    r->tune_cap[ts][a] = 0;
  }
  if (sizeof(T) == 4) {
    r->tune_plane = 1;
    r->tune_slab = 1;
  }
  const double t_default = time_apply();
  if (r->d_gmapT && sizeof(T) == 4) {
    r->tune_plane = 0;
    const double t_noplane = time_apply();
    r->tune_plane = t_noplane < t_default ? 0 : 1;
  }
  if (slab_path<T>(r)) {
    r->tune_slab = 0;
    const double t_noslab = time_apply();
    r->tune_slab = t_noslab < t_default ? 0 : 1;
  }
  const int n[3] = {g.n0, g.n1, g.n2};
  for (int a : {2, 1, 0}) {
    if (n[a] == 1) continue;
    std::vector<std::pair<int, int>> cand = {{1, 0}, {0, 0}};
    const int gl = generic_lines<T>(r, a);
    for (int c = gl / 2; c >= 1 && c >= gl / 4; c /= 2) cand.push_back({0, c});
    double best = 1e300;
    std::pair<int, int> pick = cand[0];
    for (auto& c : cand) {
      r->tune_reg[ts][a] = c.first;
      r->tune_cap[ts][a] = c.second;
      const double t = time_apply();
      if (t < best) {
        best = t;
        pick = c;
      }
    }
    r->tune_reg[ts][a] = pick.first;
    r->tune_cap[ts][a] = pick.second;
  }
  const double t_best = time_apply();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ub.release();
  yb.release();
  drop_graph(r);
  return t_default / t_best;
}

template <typename T>
static int pcg_entry(bw_rve* r, const double* k, const void* b, void* x, int nrhs, double rtol, int maxit,
                     int32_t* iters, double* relres, hipStream_t s) {
  const Geom& g = r->g;
  const double* q = qtab_for(r, k, nrhs, s);
  QTable qt = make_qtable(r, k, 1);
  const int nullv = qt.null_index[0];
  const cplx<T>* bb = (const cplx<T>*)b;
  cplx<T>* xx = (cplx<T>*)x;
  if (nullv >= 0) {
    // K is singular: b must vanish on the xi + k = 0 voxel
    std::vector<cplx<T>> vals((size_t)nrhs * 3);
    for (int v = 0; v < nrhs; ++v)
      for (int c = 0; c < 3; ++c)
        BW_HIP(hipMemcpyAsync(&vals[v * 3 + c], bb + ((size_t)v * 3 + c) * g.nvox + nullv, sizeof(cplx<T>),
                              hipMemcpyDeviceToHost, s));
    BW_HIP(hipStreamSynchronize(s));
    for (auto& z : vals)
      BW_REQUIRE(z.x == 0 && z.y == 0, BW_EINVAL, "b must vanish where xi + k = 0 (singular K)");
  }
  // x' = x * Kscale (solve the scaled system K' x' = b, K = Kscale K')
  const double ks = K_scale(r);
  scale_vectors<T>(xx, (size_t)nrhs * 3 * g.nvox, ks, s);
  PcgResult res = pcg_run<T>(r, q, qt, bb, xx, nrhs, rtol, maxit, false, s);
  scale_vectors<T>(xx, (size_t)nrhs * 3 * g.nvox, 1.0 / ks, s);
  if (nullv >= 0) zero_voxel<T>(xx, nrhs, g.nvox, nullv, s);
  BW_HIP(hipStreamSynchronize(s));
  for (int v = 0; v < nrhs; ++v) {
    if (iters) iters[v] = res.iters[v];
    if (relres) relres[v] = res.relres[v];
  }
  if (!res.converged) {
    set_error("PCG: some right-hand side did not reach the tolerance within maxit");
    return BW_ENOTCONV;
  }
  return BW_OK;
}

extern "C" int bw_pcg_solve(bw_rve* r, const double k[3], const void* b, void* x, int32_t nrhs, double rtol,
                            int32_t maxit, int32_t* iters, double* relres, void* stream) {
  BW_GUARD_BEGIN
  BW_REQUIRE(r && k, BW_EINVAL, "null argument");
  BW_REQUIRE(nrhs >= 0, BW_EINVAL, "nrhs < 0");
  BW_REQUIRE(rtol > 0 && rtol < 1, BW_EINVAL, "rtol must be in (0, 1)");
  if (nrhs == 0) return BW_OK;
  BW_REQUIRE(b && x, BW_EINVAL, "null argument");
  BW_REQUIRE(b != x, BW_EINVAL, "b and x must not alias");
  if (maxit <= 0) maxit = 20000;
  hipStream_t s = (hipStream_t)stream;
  if (r->precision == BW_FP64) return pcg_entry<double>(r, k, b, x, nrhs, rtol, maxit, iters, relres, s);
  return pcg_entry<float>(r, k, b, x, nrhs, rtol, maxit, iters, relres, s);
  BW_GUARD_END
}

extern "C" int bw_autotune(bw_rve* r, int32_t nvec, double* speedup_host, void* stream) {
  BW_GUARD_BEGIN
  BW_REQUIRE(r, BW_EINVAL, "null cell");
  BW_REQUIRE(nvec >= 1 && nvec <= 256, BW_EINVAL, "nvec out of range (1 .. 256)");
  hipStream_t s = (hipStream_t)stream;
  const double sp = r->precision == BW_FP64 ? autotune_impl<double>(r, nvec, s) : autotune_impl<float>(r, nvec, s);
  // a mixed cell's FP64 applies (Rayleigh-Ritz refinement of a few Ritz vectors)
  // get their own schedule
  if (r->precision == BW_MIXED) (void)autotune_impl<double>(r, std::min(nvec, 16), s);
  if (speedup_host) *speedup_host = sp;
  return BW_OK;
  BW_GUARD_END
}

extern "C" int bw_fft_schedule(bw_rve* r, int32_t reg[3], int32_t cap[3], int32_t set) {
  BW_GUARD_BEGIN
  BW_REQUIRE(r && reg && cap, BW_EINVAL, "null argument");
  if (set) {
    for (int a = 0; a < 3; ++a) BW_REQUIRE(cap[a] >= 0, BW_EINVAL, "tile cap must be >= 0");
    r->tune_plane = reg[0] && reg[1] ? 1 : 0;
    r->tune_slab = reg[1] && reg[2] ? 1 : 0;
    for (int t = 0; t < 2; ++t)
      for (int a = 0; a < 3; ++a) {
        r->tune_reg[t][a] = reg[a] ? 1 : 0;
        r->tune_cap[t][a] = cap[a];
      }
    drop_graph(r);
  } else {
    const int t = r->precision == BW_FP64 ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
      reg[a] = r->tune_reg[t][a];
      cap[a] = r->tune_cap[t][a];
    }
  }
  return BW_OK;
  BW_GUARD_END
}
