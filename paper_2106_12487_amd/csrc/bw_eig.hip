// Eigen-solver drivers (host side): subspace iteration (Sec. 3.3, Algorithm
// "subspace") on the batched PCG, the per-k dispersion loop (Algorithm "Full
// algorithm") with the Gamma-point deflation, and the FP64 Rayleigh-Ritz
// refinement with a-posteriori error bounds of the mixed-precision path.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <string>
#include <thread>
#include <complex>
#include <type_traits>

#include "bw_block.h"
#include "bw_internal.h"

namespace bw {

static bool verbose() {
  static const bool v = [] {
    const char* e = getenv("BW_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

struct EigOpts {
  int method, block, ncv, maxit_outer, maxit_lin, warm;
  double tol_eig, tol_lin, tol_omega;
  int kbatch;
  int precond = BW_PLAIN;
  bw_unet* net = nullptr;
  int kgroups = 1;
};

// Relative omega bound of Ritz pair p from the residual norms res[0 .. nres) of
// the Ritz pairs (M^-1 norm): Kato-Temple where the gap allows it, else the
// residual bound itself.  The gap to a neighbouring Ritz value theta_j is taken
// less that pair's own residual norm (an eigenvalue lies within res[j] of
// theta_j, whereas theta_j alone only bounds the next eigenvalue from above and
// can overstate the gap); pairs whose residual is not known (j >= nres) are not
// used, and without a known neighbour above p the residual bound is returned.
static double omega_bound(const double* res, int nres, const std::vector<double>& lam, int p) {
  const double rp = res[p];
  double gap = INFINITY;
  bool above = false;
  for (int j = 0; j < nres; ++j) {
    if (j == p) continue;
    gap = std::min(gap, std::fabs(lam[j] - lam[p]) - res[j]);
    if (j > p) above = true;
  }
  double dl = rp;
  if (above && gap > rp) dl = std::min(rp, rp * rp / gap);
  return lam[p] > 0 ? 0.5 * dl / lam[p] : dl;
}

struct Counters {
  long pcg_iters = 0, block_iters = 0, outer = 0, kap = 0, map = 0;
  long stalls = 0;   // learned inner solves that finished with the plain preconditioner
};

// Small device arrays shared by the drivers (one allocation per cell).
struct Small {
  double2 *Kq, *Mq, *Q, *dots, *coef;
  double *lam, *sc;
  int* info;
  long* vox;
  double* pol;
};

static Small small_bufs(bw_rve* r) {
  constexpr int QE = GEIG_QMAX;
  const size_t b2 = sizeof(double2);
  const size_t need = 3 * QE * QE * b2 + 2 * 256 * b2 + 2 * 256 * sizeof(double) + 64 + 256 * sizeof(long) +
                      3 * 256 * sizeof(double) + 1024;
  char* p = (char*)r->ws_misc.get(need);
  Small s;
  s.Kq = (double2*)p;
  s.Mq = s.Kq + QE * QE;
  s.Q = s.Mq + QE * QE;
  s.dots = s.Q + QE * QE;
  s.coef = s.dots + 256;
  s.lam = (double*)(s.coef + 256);
  s.sc = s.lam + 256;
  s.info = (int*)(s.sc + 256);
  s.vox = (long*)((char*)s.info + 64);
  s.pol = (double*)(s.vox + 256);
  return s;
}

// ---------------------------------------------------------------------------
// cold start: lowest plane waves of the homogeneous reference medium
// (C0, mean density): eigenpairs of P(C0, xi + k) / rho_bar per Fourier voxel.
// ---------------------------------------------------------------------------
static void eig3(double A[3][3], double w[3], double V[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = i == j;
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    if (off < 1e-300) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (std::fabs(A[p][q]) < 1e-300) continue;
        const double tau = (A[q][q] - A[p][p]) / (2 * A[p][q]);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
        const double c = 1 / std::sqrt(1 + t * t), s = t * c;
        for (int k = 0; k < 3; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 3; ++i) w[i] = A[i][i];
}

static void reference_start(const bw_rve* r, const QTable& qt, int count, std::vector<long>& vox,
                            std::vector<double>& pol) {
  const Geom& g = r->g;
  const double* q0 = qt.host.data();
  const double* q1 = q0 + g.n0;
  const double* q2 = q1 + g.n1;
  const long nv = g.nvox;
  std::vector<std::pair<double, long>> cand;
  cand.reserve(nv);
  for (long v = 0; v < nv; ++v) {
    const int i2 = (int)(v % g.n2), i1 = (int)((v / g.n2) % g.n1), i0 = (int)(v / ((long)g.n1 * g.n2));
    const double qq = q0[i0] * q0[i0] + q1[i1] * q1[i1] + q2[i2] * q2[i2];
    if (qq == 0.0) continue;
    cand.emplace_back(qq, v);
  }
  const size_t keep = std::min(cand.size(), (size_t)std::max(64, 8 * count));
  std::partial_sort(cand.begin(), cand.begin() + keep, cand.end());
  struct E {
    double lam, qq;
    long v;
    int p;
    double vec[3];
  };
  std::vector<E> es;
  double C[6][6];
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) {
      const int i = a <= b ? a * 6 - (a * (a - 1)) / 2 + (b - a) : b * 6 - (b * (b - 1)) / 2 + (a - b);
      C[a][b] = r->C0s[i];
    }
  for (size_t c = 0; c < keep; ++c) {
    const long v = cand[c].second;
    const int i2 = (int)(v % g.n2), i1 = (int)((v / g.n2) % g.n1), i0 = (int)(v / ((long)g.n1 * g.n2));
    const double qa = q0[i0], qb = q1[i1], qc = q2[i2];
    const double B[6][3] = {{qa, 0, 0}, {0, qb, 0}, {0, 0, qc}, {0, qc, qb}, {qc, 0, qa}, {qb, qa, 0}};
    double P[3][3] = {{0}};
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 6; ++a)
          for (int b = 0; b < 6; ++b) P[i][k] += B[a][i] * C[a][b] * B[b][k];
    double w[3], V[3][3];
    eig3(P, w, V);
    for (int p = 0; p < 3; ++p) es.push_back(E{w[p], cand[c].first, v, p, {V[0][p], V[1][p], V[2][p]}});
  }
  std::sort(es.begin(), es.end(), [](const E& a, const E& b) {
    if (a.lam != b.lam) return a.lam < b.lam;
    if (a.qq != b.qq) return a.qq < b.qq;
    if (a.v != b.v) return a.v < b.v;
    return a.p < b.p;
  });
  // a Gamma-like k has 3 N - 3 plane waves (the xi + k = 0 voxel carries none)
  BW_REQUIRE(count >= 0 && (size_t)count <= es.size(), BW_EINVAL,
             "more start vectors (" + std::to_string(count) + ") than reference plane waves (" +
                 std::to_string(es.size()) + ")");
  vox.resize(count);
  pol.resize(3 * count);
  for (int i = 0; i < count; ++i) {
    vox[i] = es[i].v;
    for (int c = 0; c < 3; ++c) pol[3 * i + c] = es[i].vec[c];
  }
}

// The entries written by launch_set_entries must address distinct elements (one
// thread per element): checked on the host lists before they are uploaded.
static void require_distinct_entries(const std::vector<long>& vec, const std::vector<long>& vox) {
  std::vector<std::pair<long, long>> pr(vec.size());
  for (size_t i = 0; i < vec.size(); ++i) pr[i] = {vec[i], vox[i]};
  std::sort(pr.begin(), pr.end());
  BW_REQUIRE(std::adjacent_find(pr.begin(), pr.end()) == pr.end(), BW_EINVAL,
             "internal: two start-vector entries address the same element");
}

// ---------------------------------------------------------------------------
// per-k subspace iteration
// ---------------------------------------------------------------------------
struct KOut {
  std::vector<double> lam;   // n_want scaled eigenvalues (ascending)
  std::vector<double> bound; // relative bound on omega
  int n_want = 0;
  long jstar = -1;
  bool converged = true;
  int outer = 0;
};

template <typename T> static void apply_K_blk(bw_rve* r, const double* dq, const cplx<T>* u, cplx<T>* y, int nv,
                                               Counters& c, hipStream_t s) {
  if (nv <= 0) return;
  launch_apply_K<T>(r, dq, u, y, nv, 1.0, ws<T>(r).work((size_t)nv * 6 * r->g.nvox), s);
  c.kap += nv;
}
template <typename T> static void apply_M_blk(bw_rve* r, const cplx<T>* u, cplx<T>* y, int nv, bool inverse,
                                               Counters& c, hipStream_t s) {
  if (nv <= 0) return;
  if (r->rho_unit) {   // one density: M' and its inverse are the identity
    BW_HIP(hipMemcpyAsync(y, u, (size_t)nv * 3 * r->g.nvox * sizeof(cplx<T>), hipMemcpyDeviceToDevice, s));
  } else {
    launch_apply_Minv_or_M<T>(r, u, y, nv, inverse, ws<T>(r).work((size_t)nv * 6 * r->g.nvox), s);
  }
  c.map += nv;
}

// Rigid-translation data at a Gamma-like k: MN = M e_{j*, c}, c = 0..2.
template <typename T>
static void rigid_MN(bw_rve* r, long jstar, cplx<T>* N, cplx<T>* MN, Small& sm, Counters& c, hipStream_t s) {
  std::vector<long> vox = {jstar, jstar, jstar};
  std::vector<double> pol = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  h2d(sm.vox, vox.data(), 3 * sizeof(long), s);
  h2d(sm.pol, pol.data(), 9 * sizeof(double), s);
  launch_planewaves<T>(N, 3, r->g.nvox, sm.vox, sm.pol, s);
  apply_M_blk<T>(r, N, MN, 3, false, c, s);
  BW_HIP(hipStreamSynchronize(s));
}

// FP64 Rayleigh-Ritz on span(U) and residual bounds (M^-1 norm).  U is
// replaced by the Ritz vectors.  Returns lam (q) and the relative omega bound
// of the first n_want.
static void rr64_bounds(bw_rve* r, const double* dq, cplx<double>*& U, int q, int n_want, std::vector<double>& lam,
                        std::vector<double>& bound, bool do_rr, const cplx<double>* KUin, const cplx<double>* MUin,
                        Counters& cnt, hipStream_t s) {
  Workspace<double>& w = ws<double>(r);
  const long n3 = r->g.nvox * 3;
  Small sm = small_bufs(r);
  const cplx<double>* KU = KUin;
  const cplx<double>* MU = MUin;
  cplx<double>* R = w.vec(9, (size_t)q * n3);
  cplx<double>* Z = w.vec(11, (size_t)q * n3);
  lam.resize(q);
  // residuals of the wanted pairs and of the next one (its gap enters the bound)
  const int nr = n_want > 0 ? std::min(q, n_want + 1) : 0;
  // M' = I (one density): M U is U and M^-1 R is R, no copies
  const bool unit = r->rho_unit != 0;
  if (do_rr) {
    cplx<double>* U2 = w.vec(4, (size_t)q * n3);
    cplx<double>* KU0 = w.vec(5, (size_t)q * n3);
    cplx<double>* MU0 = unit ? U : w.vec(6, (size_t)q * n3);
    cplx<double>* KU1 = w.vec(7, (size_t)q * n3);
    cplx<double>* MU1 = unit ? U2 : w.vec(8, (size_t)q * n3);
    apply_K_blk<double>(r, dq, U, KU0, q, cnt, s);
    if (!unit) apply_M_blk<double>(r, U, MU0, q, false, cnt, s);
    launch_gram<double>(U, q, KU0, q, n3, n3, sm.Kq, r->ws_red, r->d_ctr, s);
    launch_gram<double>(U, q, MU0, q, n3, n3, sm.Mq, r->ws_red, r->d_ctr, s);
    launch_small_geig(sm.Kq, sm.Mq, q, sm.lam, sm.Q, sm.info, s);
    launch_ritz<double>(U, q, sm.Q, q, U2, q, n3, n3, s);
    launch_ritz<double>(KU0, q, sm.Q, q, KU1, nr, n3, n3, s);
    if (!unit) launch_ritz<double>(MU0, q, sm.Q, q, MU1, nr, n3, n3, s);
    std::swap(w.v[3], w.v[4]);
    U = (cplx<double>*)w.v[3].p;
    KU = KU1;
    MU = unit ? U : MU1;
  } else {
    h2d(sm.lam, lam.data(), q * sizeof(double), s);
  }
  launch_lincomb<double>(KU, MU, sm.lam, R, nr, n3, n3, s);
  if (!unit) apply_M_blk<double>(r, R, Z, nr, true, cnt, s);
  launch_dots<double>(R, unit ? R : Z, nr, n3, n3, sm.dots, r->ws_red, r->d_ctr + 64, s);
  std::vector<double2> rn(nr);
  int info = 0;
  if (do_rr) {
    BW_HIP(hipMemcpyAsync(lam.data(), sm.lam, q * sizeof(double), hipMemcpyDeviceToHost, s));
    BW_HIP(hipMemcpyAsync(&info, sm.info, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  if (nr > 0) BW_HIP(hipMemcpyAsync(rn.data(), sm.dots, nr * sizeof(double2), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  BW_REQUIRE(info == 0, BW_EINVAL, "Rayleigh-Ritz Gram matrix not positive definite");
  std::vector<double> res(nr);
  for (int p = 0; p < nr; ++p) res[p] = std::sqrt(std::max(rn[p].x, 0.0));
  bound.assign(n_want, 0.0);
  for (int p = 0; p < n_want; ++p) bound[p] = omega_bound(res.data(), nr, lam, p);
}

// FP64 refinement of a block of Ritz vectors (mixed-precision path): FP64
// Rayleigh-Ritz and residual R = K U - lambda M U, then, while a bound misses
// the target, an FP32 correction solve K D = R (iterative refinement driven by
// the FP64 residual; U - D is one step of inverse iteration) and a new FP64
// Rayleigh-Ritz.  U64 (q vectors, FP64 workspace slot 3) is updated in place.
template <typename T>
static void refine64(bw_rve* r, const double* dq, const QTable& qt, long jstar, int q, int n_want,
                     std::vector<double>& lam, std::vector<double>& bound, double target, int rounds, Counters& cnt,
                     hipStream_t s) {
  const long n3 = r->g.nvox * 3;
  Small sm = small_bufs(r);
  Workspace<double>& w64 = ws<double>(r);
  cplx<double>* U64 = (cplx<double>*)w64.v[3].p;
  rr64_bounds(r, dq, U64, q, n_want, lam, bound, true, nullptr, nullptr, cnt, s);
  for (int it = 0; it < rounds && n_want > 0; ++it) {
    const double worst = *std::max_element(bound.begin(), bound.end());
    if (verbose()) fprintf(stderr, "[bw]   refinement round %d: worst bound %.3e\n", it, worst);
    if (worst <= target) break;
    const cplx<double>* R = (const cplx<double>*)w64.v[9].p;  // K U - lambda M U (first n_want)
    Workspace<T>& w = ws<T>(r);
    cplx<T>* Rt = w.vec(12, (size_t)n_want * n3);
    cplx<T>* D = w.vec(13, (size_t)n_want * n3);
    if (sizeof(T) == 4)
      launch_convert<double, float>(R, (cplx<float>*)Rt, (size_t)n_want * n3, s);
    else
      BW_HIP(hipMemcpyAsync(Rt, R, (size_t)n_want * n3 * sizeof(cplx<T>), hipMemcpyDeviceToDevice, s));
    // At a Gamma-like k, K D = R is solvable only for the part of R orthogonal to
    // null(K) (the rigid translations, i.e. the xi + k = 0 coefficients).  R has a
    // component there at the rounding level of the block's M-orthogonality to the
    // translations, which the preconditioned iteration cannot reduce (P^ is zero
    // at that voxel): left in, it holds the residual above the tolerance until maxit.
    if (jstar >= 0) zero_voxel<T>(Rt, n_want, r->g.nvox, jstar, s);
    BW_HIP(hipMemsetAsync(D, 0, (size_t)n_want * n3 * sizeof(cplx<T>), s));
    PcgResult pr = pcg_run<T>(r, dq, qt, Rt, D, n_want, sizeof(T) == 4 ? 1e-6 : 1e-10, 2000, true, s, false, false);
    cnt.pcg_iters += pr.total_iters;
    cnt.block_iters += pr.block_iters;
    cnt.kap += pr.k_applies;
    cplx<double>* D64 = w64.vec(12, (size_t)n_want * n3);
    if (sizeof(T) == 4)
      launch_convert<float, double>((const cplx<float>*)D, D64, (size_t)n_want * n3, s);
    else
      BW_HIP(hipMemcpyAsync(D64, D, (size_t)n_want * n3 * sizeof(cplx<double>), hipMemcpyDeviceToDevice, s));
    if (jstar >= 0) {  // keep the block M-orthogonal to the rigid translations
      cplx<double>* MD = w64.vec(13, (size_t)n_want * n3);
      cplx<double>* MN = w64.vec(14, (size_t)3 * n3);
      cplx<double>* N3 = w64.vec(15, (size_t)3 * n3);
      rigid_MN<double>(r, jstar, N3, MN, sm, cnt, s);
      apply_M_blk<double>(r, D64, MD, n_want, false, cnt, s);
      launch_deflate<double>(D64, MD, MN, n_want, r->g.nvox, jstar, sm.coef, s);
    }
    std::vector<double> ones(n_want, 1.0);
    h2d(sm.sc, ones.data(), n_want * sizeof(double), s);
    U64 = (cplx<double>*)w64.v[3].p;
    launch_lincomb<double>(U64, D64, sm.sc, U64, n_want, n3, n3, s);  // U <- U - D
    BW_HIP(hipStreamSynchronize(s));
    rr64_bounds(r, dq, U64, q, n_want, lam, bound, true, nullptr, nullptr, cnt, s);
  }
}

template <typename T>
static KOut subspace_k(bw_rve* r, const double* k, int nmodes, int q, const EigOpts& o, bool& have_start,
                       std::vector<double>& lam_prev, Counters& cnt, hipStream_t s) {
  const Geom& g = r->g;
  const long n3 = g.nvox * 3;
  Workspace<T>& w = ws<T>(r);
  Small sm = small_bufs(r);
  KOut out;
  std::vector<double> ks((size_t)q * 3);
  for (int v = 0; v < q; ++v)
    for (int a = 0; a < 3; ++a) ks[3 * v + a] = k[a];
  QTable qt = make_qtable(r, ks.data(), q);
  const double* dq = upload_qtable(r, qt, r->ws_q2, s);
  out.jstar = qt.null_index[0];
  out.n_want = nmodes - (out.jstar >= 0 ? 3 : 0);
  const int nw = out.n_want;
  BW_REQUIRE(nw >= 0 && nw < q, BW_EINVAL, "block must exceed the number of wanted modes");
  cplx<T>* U = w.vec(3, (size_t)q * n3);
  cplx<T>* Ub = w.vec(4, (size_t)q * n3);
  cplx<T>* V = w.vec(5, (size_t)q * n3);
  cplx<T>* MUb = w.vec(6, (size_t)q * n3);
  cplx<T>* KU = w.vec(7, (size_t)q * n3);
  cplx<T>* MU = w.vec(8, (size_t)q * n3);
  cplx<T>* R = w.vec(9, (size_t)q * n3);
  cplx<T>* MN = w.vec(10, (size_t)3 * n3);
  if (out.jstar >= 0) rigid_MN<T>(r, out.jstar, R, MN, sm, cnt, s);
  if (!have_start) {
    std::vector<long> vox;
    std::vector<double> pol;
    reference_start(r, qt, q, vox, pol);
    h2d(sm.vox, vox.data(), q * sizeof(long), s);
    h2d(sm.pol, pol.data(), 3 * q * sizeof(double), s);
    launch_planewaves<T>(U, q, g.nvox, sm.vox, sm.pol, s);
    BW_HIP(hipStreamSynchronize(s));
    lam_prev.clear();
  } else if (q >= nw + 3) {
    // warm start: the block's tail (beyond the wanted modes and two more) also gets
    // the lowest reference plane waves of this k added, so that directions absent
    // from the previous k's Ritz block enter; for a homogeneous cell the plane waves
    // are exact eigenvectors, and no iteration would bring a missing one in
    const int keep = nw + 2, nf = q - keep;
    std::vector<long> vox, vec(nf);
    std::vector<double> pol;
    reference_start(r, qt, nf, vox, pol);
    for (int i = 0; i < nf; ++i) vec[i] = keep + i;
    require_distinct_entries(vec, vox);
    h2d(sm.vox, vox.data(), nf * sizeof(long), s);
    h2d(sm.vox + 128, vec.data(), nf * sizeof(long), s);
    h2d(sm.pol, pol.data(), 3 * nf * sizeof(double), s);
    launch_set_entries<T>(U, n3, g.nvox, nf, sm.vox + 128, sm.vox, sm.pol, s, true);
    BW_HIP(hipStreamSynchronize(s));
  }
  const bool fp32 = sizeof(T) == 4;
  // FP32 stage: the eigenvalue change must settle to tol (at least 1e-6) and the
  // residual err2 must either reach 10 tol or stop improving (it floors at the
  // FP32 round-off of K, about eps * lambda_max / lambda); the FP64
  // Rayleigh-Ritz step and its bounds then decide the accuracy.
  const double tol = fp32 ? std::max(o.tol_eig, 1e-6) : o.tol_eig;
  const double tol_lin = fp32 ? std::max(o.tol_lin, 1e-6) : o.tol_lin;
  const double bound_target = o.tol_omega > 0 ? o.tol_omega : 5.0 * o.tol_eig;
  std::vector<double> lam(q), lam_old, inv(q), err2_hist;
  bool conv = false;
  int it = 0;
  int round = 0;
  // After the first iteration at this k the Ritz step already provides M U
  // (next right-hand sides) and R = K U - lambda M U for the whole block, so the
  // PCG initial residual for x0 = U / lambda is -R / lambda: no extra applies.
  bool have_KU = false;
  std::vector<double> ninv(q);
  for (; it < o.maxit_outer; ++it) {
    if (have_KU) {
      std::swap(V, MU);                          // v_p = M U_p from the Ritz step
    } else {
      apply_M_blk<T>(r, U, V, q, false, cnt, s);  // v_p = M U_p
      if (out.jstar >= 0) launch_deflate<T>(U, V, MN, q, g.nvox, out.jstar, sm.coef, s);
    }
    const bool warm = (int)lam_prev.size() == q;
    bool r_ready = false;
    if (warm) {
      for (int p = 0; p < q; ++p) {
        inv[p] = lam_prev[p] > 0 ? 1.0 / lam_prev[p] : 0.0;
        ninv[p] = -inv[p];
      }
      h2d(sm.sc, inv.data(), q * sizeof(double), s);
      launch_scale_cols<T>(U, sm.sc, Ub, q, n3, n3, s);  // x0 = U / lambda
      if (have_KU) {
        h2d(sm.sc + 128, ninv.data(), q * sizeof(double), s);
        launch_scale_cols<T>(R, sm.sc + 128, w.vec(0, (size_t)q * n3), q, n3, n3, s);  // r0 = -R / lambda
        r_ready = true;
      }
    } else {
      BW_HIP(hipMemsetAsync(Ub, 0, (size_t)q * n3 * sizeof(cplx<T>), s));
    }
    double tl = tol_lin;
    if (o.tol_omega > 0) tl = std::max(tol_lin, std::min(1e-2, err2_hist.empty() ? 1e-3 : 0.05 * err2_hist.back()));
    // Ubar = K^-1 v; the outer residual check uses the true K, so the inner
    // solve stops on its recurrence residual
    PcgResult pr = pcg_run<T>(r, dq, qt, V, Ub, q, tl, o.maxit_lin, !warm, s, r_ready, false);
    cnt.pcg_iters += pr.total_iters;
    cnt.block_iters += pr.block_iters;
    cnt.kap += pr.k_applies;
    apply_M_blk<T>(r, Ub, MUb, q, false, cnt, s);
    if (out.jstar >= 0) launch_deflate<T>(Ub, MUb, MN, q, g.nvox, out.jstar, sm.coef, s);
    launch_gram<T>(Ub, q, V, q, n3, n3, sm.Kq, r->ws_red, r->d_ctr, s);    // Kq = Ubar^H Kn
    launch_gram<T>(Ub, q, MUb, q, n3, n3, sm.Mq, r->ws_red, r->d_ctr, s);  // Mq = Ubar^H Mn
    launch_small_geig(sm.Kq, sm.Mq, q, sm.lam, sm.Q, sm.info, s);
    launch_ritz<T>(Ub, q, sm.Q, q, U, q, n3, n3, s);                       // U = Ubar Q
    launch_ritz<T>(MUb, q, sm.Q, q, MU, q, n3, n3, s);                     // M U
    apply_K_blk<T>(r, dq, U, KU, q, cnt, s);
    launch_lincomb<T>(KU, MU, sm.lam, R, q, n3, n3, s);                    // R = K U - lambda M U
    have_KU = true;
    const int nr = std::min(q, nw + 1);   // the wanted pairs and the next one
    launch_dots<T>(R, R, nr, n3, n3, sm.dots, r->ws_red, r->d_ctr + 64, s);
    launch_dots<T>(MU, MU, nr, n3, n3, sm.dots + 128, r->ws_red2, r->d_ctr + 320, s);
    std::vector<double2> rr(nr), mm(nr);
    int info = 0;
    BW_HIP(hipMemcpyAsync(lam.data(), sm.lam, q * sizeof(double), hipMemcpyDeviceToHost, s));
    BW_HIP(hipMemcpyAsync(&info, sm.info, sizeof(int), hipMemcpyDeviceToHost, s));
    if (nw > 0) {
      BW_HIP(hipMemcpyAsync(rr.data(), sm.dots, nr * sizeof(double2), hipMemcpyDeviceToHost, s));
      BW_HIP(hipMemcpyAsync(mm.data(), sm.dots + 128, nr * sizeof(double2), hipMemcpyDeviceToHost, s));
    }
    BW_HIP(hipStreamSynchronize(s));
    BW_REQUIRE(info == 0, BW_EINVAL, "subspace Gram matrix lost positive definiteness (block rank deficient)");
    double err1 = INFINITY, err2 = 0;
    if (!lam_old.empty()) {
      double num = 0, den = 0;
      for (int p = 0; p < nw; ++p) {
        num += (lam[p] - lam_old[p]) * (lam[p] - lam_old[p]);
        den += lam_old[p] * lam_old[p];
      }
      err1 = den > 0 ? std::sqrt(num / den) : 0.0;
    }
    for (int p = 0; p < nw; ++p)
      err2 = std::max(err2, std::sqrt(std::max(rr[p].x, 0.0)) / (lam[p] * std::sqrt(std::max(mm[p].x, 1e-300))));
    err2_hist.push_back(err2);
    lam_old = lam;
    lam_prev = lam;
    have_start = true;
    cnt.outer += 1;
    if (verbose())
      fprintf(stderr, "[bw] k=(%.4g,%.4g,%.4g) outer %d err1 %.3e err2 %.3e pcg %ld (block %ld) lam0 %.6e\n", k[0],
              k[1], k[2], it, err1, err2, pr.total_iters, pr.block_iters, lam[0]);
    const size_t h = err2_hist.size();
    const bool stalled = fp32 && h >= 4 && err2 > 0.8 * err2_hist[h - 4];
    // bound-based test: ||r||_{M^-1} <= ||r|| / sqrt(min rho') for M-normalized Ritz vectors
    bool bounds_ok = false;
    if (o.tol_omega > 0 && nw > 0) {
      double worst = 0;
      std::vector<double> res(nr);
      for (int p = 0; p < nr; ++p) res[p] = std::sqrt(std::max(rr[p].x, 0.0) / r->rho_min_s);
      for (int p = 0; p < nw; ++p) worst = std::max(worst, omega_bound(res.data(), nr, lam, p));
      bounds_ok = worst <= o.tol_omega && std::isfinite(err1);
    }
    const bool rule = o.tol_omega > 0 ? (bounds_ok || (fp32 && stalled && err1 <= tol))
                                      : (err1 <= tol && (err2 <= 10.0 * tol || stalled));
    if (nw == 0 || rule) {
      if (!fp32 || nw == 0) {
        conv = true;
        ++it;
        break;
      }
      // FP64 Rayleigh-Ritz on the FP32 block, FP64-residual-driven refinement and the bounds
      std::vector<double> lam64, bnd;
      Workspace<double>& w64 = ws<double>(r);
      cplx<double>* U64 = w64.vec(3, (size_t)q * n3);
      launch_convert<float, double>((const cplx<float>*)U, U64, (size_t)q * n3, s);
      refine64<T>(r, dq, qt, out.jstar, q, nw, lam64, bnd, bound_target, 3, cnt, s);
      U64 = (cplx<double>*)w64.v[3].p;
      launch_convert<double, float>(U64, (cplx<float>*)U, (size_t)q * n3, s);
      lam_prev = lam64;
      have_KU = false;
      lam_old.clear();
      err2_hist.clear();
      out.lam.assign(lam64.begin(), lam64.begin() + nw);
      out.bound = bnd;
      const double worst = *std::max_element(bnd.begin(), bnd.end());
      if (verbose()) fprintf(stderr, "[bw]   FP64 Rayleigh-Ritz: worst bound %.3e\n", worst);
      if (worst <= bound_target || ++round >= 4) {
        conv = worst <= bound_target;
        ++it;
        break;
      }
    }
  }
  out.outer = it;
  out.converged = conv;
  if (nw > 0 && !fp32) {
    std::vector<double> lam64 = lam, bnd;
    cplx<double>* Ud = (cplx<double>*)U;
    rr64_bounds(r, dq, Ud, q, nw, lam64, bnd, false, (const cplx<double>*)KU, (const cplx<double>*)MU, cnt, s);
    out.lam.assign(lam64.begin(), lam64.begin() + nw);
    out.bound = bnd;
  } else if (nw > 0 && out.lam.empty()) {
    // FP32 stage hit maxit before its Rayleigh-Ritz step
    std::vector<double> lam64, bnd;
    cplx<double>* U64 = ws<double>(r).vec(3, (size_t)q * n3);
    launch_convert<float, double>((const cplx<float>*)U, U64, (size_t)q * n3, s);
    rr64_bounds(r, dq, U64, q, nw, lam64, bnd, true, nullptr, nullptr, cnt, s);
    out.lam.assign(lam64.begin(), lam64.begin() + nw);
    out.bound = bnd;
  }
  return out;
}

// ---------------------------------------------------------------------------
// modes output (SI M-normalization: U_SI = U' / sqrt(rho_bar))
// ---------------------------------------------------------------------------
template <typename T>
static void write_modes(bw_rve* r, const KOut& ko, int nmodes, void* modes, int kidx, hipStream_t s) {
  if (!modes) return;
  const long n3 = r->g.nvox * 3;
  cplx<T>* dst = (cplx<T>*)modes + (size_t)kidx * nmodes * n3;
  Small sm = small_bufs(r);
  int off = 0;
  const double a = 1.0 / std::sqrt(r->rho_bar);
  std::vector<long> vox = {ko.jstar, ko.jstar, ko.jstar};
  std::vector<double> pol = {a, 0, 0, 0, a, 0, 0, 0, a};
  std::vector<double> sc(std::max(ko.n_want, 1), a);
  if (ko.jstar >= 0) {
    h2d(sm.vox, vox.data(), 3 * sizeof(long), s);
    h2d(sm.pol, pol.data(), 9 * sizeof(double), s);
    launch_planewaves<T>(dst, 3, r->g.nvox, sm.vox, sm.pol, s);
    off = 3;
  }
  if (ko.n_want > 0) {
    // the FP64 Ritz block (refined) lives in the FP64 workspace slot 3 for both paths
    const cplx<double>* U = (const cplx<double>*)ws<double>(r).v[3].p;
    h2d(sm.sc, sc.data(), ko.n_want * sizeof(double), s);
    if (sizeof(T) == 8) {
      launch_scale_cols<double>(U, sm.sc, (cplx<double>*)(dst + (size_t)off * n3), ko.n_want, n3, n3, s);
    } else {
      cplx<double>* tmp = ws<double>(r).vec(4, (size_t)ko.n_want * n3);
      launch_scale_cols<double>(U, sm.sc, tmp, ko.n_want, n3, n3, s);
      launch_convert<double, float>(tmp, (cplx<float>*)(dst + (size_t)off * n3), (size_t)ko.n_want * n3, s);
    }
  }
  BW_HIP(hipStreamSynchronize(s));
}

// 64-bit seed from the bits of a wave vector (splitmix64 finalizer per component).
static unsigned long long wave_vector_seed(const double* k) {
  unsigned long long h = 0x2106124870ULL;
  for (int a = 0; a < 3; ++a) {
    unsigned long long b;
    std::memcpy(&b, k + a, sizeof(b));
    h = (h ^ b) + 0x9e3779b97f4a7c15ULL;
    h = (h ^ (h >> 30)) * 0xbf58476d1ce4e5b9ULL;
    h = (h ^ (h >> 27)) * 0x94d049bb133111ebULL;
    h ^= h >> 31;
  }
  return h;
}

// Host side of the delayed re-orthogonalization of Lanczos step j (one wave
// vector; H is the m x m projected matrix, row-major).  Inputs: d1[i] = <v_i,
// v~_j>_M for i <= j (v~_j: the pending vector, orthogonalized once) and d2[i] =
// <v_i, X>_M with X = OP v~_j.  With s = d1[0..j-1] and nu^2 = d1[j] - |s|^2 the
// finished vector is v_j = (v~_j - V s) / nu.  The relation OP V = V H + v~_j h_j^T
// (h_j: row j of H) then reads OP V = V (H + s h_j^T) + v_j nu h_j^T, and
// OP v_j = (X - V t - v_j tau) / nu with t = H[0..j-1, 0..j-1] s, tau = h_j s (both
// after the update); its products with the finished basis are c_i = (d2_i - t_i) / nu
// and c_j = ((d2_j - s^H d2) / nu - tau) / nu.  Writes column j of H (real parts:
// the projected matrix of the Hermitian OP is real symmetric up to rounding) and the
// coefficients of the update kernel: a = s / nu, b = t / nu + c, f0 = f1 = 1 / nu,
// g = tau / nu + c_j.
static void delayed_reorth_coefficients(double* H, int m, int j, const double2* d1, const double2* d2,
                                        double2* coef) {
  using C = std::complex<double>;
  std::vector<C> sv(j), z(j), t(j, 0.0);
  double ss = 0.0;
  for (int i = 0; i < j; ++i) {
    sv[i] = C(d1[i].x, d1[i].y);
    z[i] = C(d2[i].x, d2[i].y);
    ss += std::norm(sv[i]);
  }
  const double om = d1[j].x;
  const double nu = std::sqrt(std::max(om - ss, 1e-12 * std::max(om, 1e-300)));
  for (int l = 0; l < j; ++l) {
    const double hjl = H[(size_t)j * m + l];
    if (hjl == 0.0) continue;
    for (int i = 0; i < j; ++i) H[(size_t)i * m + l] += sv[i].real() * hjl;
    H[(size_t)j * m + l] = nu * hjl;
    for (int i = 0; i < j; ++i) H[(size_t)l * m + i] = H[(size_t)i * m + l];
    H[(size_t)l * m + j] = H[(size_t)j * m + l];
  }
  C tau = 0.0, sz = 0.0;
  for (int l = 0; l < j; ++l) {
    tau += H[(size_t)j * m + l] * sv[l];
    sz += std::conj(sv[l]) * z[l];
  }
  for (int i = 0; i < j; ++i)
    for (int l = 0; l < j; ++l) t[i] += H[(size_t)i * m + l] * sv[l];
  const C cj = ((C(d2[j].x, d2[j].y) - sz) / nu - tau) / nu;
  for (int i = 0; i < j; ++i) {
    const C ci = (z[i] - t[i]) / nu;
    const C a = sv[i] / nu, b = t[i] / nu + ci;
    coef[i] = make_double2(a.real(), a.imag());
    coef[j + i] = make_double2(b.real(), b.imag());
    H[(size_t)i * m + j] = ci.real();
    H[(size_t)j * m + i] = ci.real();
  }
  H[(size_t)j * m + j] = cj.real();
  const C g = tau / nu + cj;
  coef[2 * j] = make_double2(1.0 / nu, 0.0);
  coef[2 * j + 1] = make_double2(1.0 / nu, 0.0);
  coef[2 * j + 2] = make_double2(g.real(), g.imag());
}

// ---------------------------------------------------------------------------
// batched thick-restart shift-invert Lanczos (Sec. 3.3, implicitly restarted
// Lanczos on the shifted-inverse operator).  Every wave vector of the batch
// runs its own Lanczos process on OP = K(k)^-1 M in the M inner product with
// full re-orthogonalization; the solves of one Lanczos step of all of them
// share one batched PCG (one right-hand side per wave vector).  A restart
// keeps the leading Ritz vectors and the residual direction (thick restart:
// the same subspace as implicit restarts with the unwanted Ritz values as
// exact shifts).  Converged wave vectors leave the batch.
// ---------------------------------------------------------------------------
// Results of wave vector k of the batch go to output row kmap[k] (kmap null:
// kofs + k).
template <typename T>
static int lanczos_batch(bw_rve* r, const double* k_list, int nk, int nmodes, const EigOpts& o, double* omega,
                         double* err, void* modes, int kofs, Counters& cnt, hipStream_t s,
                         const int* kmap = nullptr) {
  const Geom& g = r->g;
  const long n3 = g.nvox * 3;
  Small sm = small_bufs(r);
  const bool fp32 = sizeof(T) == 4;
  QTable qt = make_qtable(r, k_list, nk);
  const double* dq = upload_qtable(r, qt, r->ws_q2, s);
  // a cell group: wave vector k of the batch (and its vector in every batched
  // launch) belongs to cell kcell[k]; the per-k steps (start vector, rigid modes,
  // FP64 refinement and bounds) select that cell alone
  const bool grouped = r->ncell > 1;
  CellSel bsel;
  std::vector<int> kcell(nk, 0);
  const std::vector<double> C0s_first(r->C0s, r->C0s + 21);
  const double rho_min_all = r->rho_min_s;
  if (grouped) {
    BW_REQUIRE((int)r->kcell_bounds.size() == r->ncell + 1, BW_EINVAL, "cell group without wave-vector bounds");
    bsel.n = r->ncell;
    bsel.gstride = g.nvox;
    bsel.c0tab32 = r->d_C0tab32;
    bsel.c0tab64 = r->d_C0tab64;
    for (int i = 0; i + 1 < r->ncell; ++i) bsel.bound[i] = (int)std::max(0L, r->kcell_bounds[i + 1] - (long)kofs);
    for (int k = 0; k < nk; ++k) kcell[k] = bsel.cell(k);
  }
  auto select_cell = [&](int c) {
    if (!grouped) return;
    CellSel u = bsel;
    u.n = c + 1;
    for (int i = 0; i < c; ++i) u.bound[i] = 0;
    r->csel = u;
    std::copy(r->cell_C0s.begin() + 21 * c, r->cell_C0s.begin() + 21 * (c + 1), r->C0s);
    r->rho_min_s = r->cell_rho_min[c];
  };
  auto select_batch = [&]() {
    if (!grouped) return;
    r->csel = bsel;
    std::copy(C0s_first.begin(), C0s_first.end(), r->C0s);
    r->rho_min_s = rho_min_all;
  };
  struct Restore {   // the handle leaves in its one-cell state, also on errors
    bw_rve* r;
    std::vector<double> c0;
    double rm;
    ~Restore() {
      r->csel = CellSel{};
      std::copy(c0.begin(), c0.end(), r->C0s);
      r->rho_min_s = rm;
    }
  } restore{r, C0s_first, rho_min_all};
  select_batch();
  std::vector<int> nwk(nk);
  int nwmax = 0;
  for (int k = 0; k < nk; ++k) {
    nwk[k] = nmodes - (qt.null_index[k] >= 0 ? 3 : 0);
    nwmax = std::max(nwmax, nwk[k]);
  }
  const int m = o.ncv > 0 ? o.ncv : std::max(2 * nwmax + 1, 20);
  BW_REQUIRE(m <= GEIG_QMAX && m >= nwmax + 2, BW_EINVAL, "ncv must satisfy nmodes + 2 <= ncv <= 48");
  // the Krylov space of K^-1 M (rigid translations removed) has at most 3 N - 3
  // dimensions: a longer basis would break down and fill with rounding noise
  BW_REQUIRE((long)m <= 3L * g.nvox - 3, BW_EINVAL,
             "the Lanczos basis (ncv = " + std::to_string(m) +
                 " vectors) exceeds the cell's degrees of freedom less 3; use the subspace method");
  const int kk = std::min({m - 1, nwmax + (m - nwmax) / 2, GRAM_QMAX});  // vectors kept at a restart
  const int qsel = std::min(m, nwmax + 2);                                // Ritz vectors refined in FP64
  Workspace<T>& w = wl<T>(r);
  const long xk = (long)(m + 1) * n3;
  cplx<T>* V = w.vec(0, (size_t)nk * xk);
  // with M' = I the basis is its own M-image: no second basis to store or restart
  const bool unit = r->rho_unit != 0;
  cplx<T>* MV = unit ? V : w.vec(1, (size_t)nk * xk);
  // a restart writes the kept Ritz vectors of every restarting wave vector into a
  // second basis, and the two bases swap roles (no copy back)
  cplx<T>* V2 = w.vec(12, (size_t)nk * xk);
  cplx<T>* MV2 = unit ? V2 : w.vec(13, (size_t)nk * xk);
  cplx<T>* B = w.vec(2, (size_t)nk * n3);
  cplx<T>* X = w.vec(3, (size_t)nk * n3);
  cplx<T>* MF = w.vec(4, (size_t)nk * n3);
  cplx<T>* TMP = w.vec(5, (size_t)qsel * n3);
  cplx<T>* MN = w.vec(6, (size_t)3 * n3);
  cplx<T>* N3 = w.vec(7, (size_t)3 * n3);
  const size_t hcount = (size_t)nk * (m + 1);
  const int ldc = 2 * (m + 1) + 3;  // coefficients of the re-orthogonalization update per wave vector
  char* sb = (char*)w.v[8].get((2 * hcount + (size_t)nk * ldc) * sizeof(double2) +
                               nk * (sizeof(double) + sizeof(int)) + 1024);
  double2* hd = (double2*)sb;
  double2* hd2 = hd + hcount;
  double2* cfd = hd2 + hcount;
  double* scd = (double*)(cfd + (size_t)nk * ldc);
  int* actd = (int*)(scd + nk);
  long jcache = -1;
  int ccache = -1;
  auto ensure_MN = [&](long j, int c) {
    if (j != jcache || c != ccache) {
      select_cell(c);
      rigid_MN<T>(r, j, N3, MN, sm, cnt, s);
      select_batch();
      jcache = j;
      ccache = c;
    }
  };
  auto deflate_batch = [&](cplx<T>* Xb, cplx<T>* MXb, const std::vector<int>& act) {
    for (int k = 0; k < nk; ++k)
      if (act[k] && qt.null_index[k] >= 0) {
        ensure_MN(qt.null_index[k], kcell[k]);
        launch_deflate<T>(Xb + (size_t)k * n3, MXb + (size_t)k * n3, MN, 1, g.nvox, qt.null_index[k], sm.coef, s);
      }
  };
  std::vector<int> act(nk, 1);
  std::vector<double> sc(nk), beta(nk, 0.0), tolk(nk), best(nk, INFINITY);
  for (int k = 0; k < nk; ++k) tolk[k] = fp32 ? std::max(o.tol_omega > 0 ? o.tol_omega : o.tol_eig, 1e-6)
                                               : (o.tol_omega > 0 ? o.tol_omega : o.tol_eig);
  const double bound_target = o.tol_omega > 0 ? o.tol_omega : 5.0 * o.tol_eig;
  const double lscale = r->Cref / (r->rho_bar * r->ell * r->ell);
  auto upload_act = [&]() { h2d(actd, act.data(), nk * sizeof(int), s); };
  auto upload_sc = [&]() { h2d(scd, sc.data(), nk * sizeof(double), s); };

  // start vectors: the lowest reference plane wave plus a little of the next three
  BW_HIP(hipMemsetAsync(B, 0, (size_t)nk * n3 * sizeof(cplx<T>), s));
  {
    std::vector<long> vec, vox;
    std::vector<double> val;
    for (int k = 0; k < nk; ++k) {
      QTable q1 = make_qtable(r, k_list + 3 * k, 1);
      std::vector<long> vx;
      std::vector<double> pl;
      select_cell(kcell[k]);
      reference_start(r, q1, 4, vx, pl);
      select_batch();
      // plane waves at one voxel (several polarizations of one wave) are summed
      // here, so that every element of B is written by one thread only
      const size_t first = vox.size();
      for (size_t e = 0; e < vx.size(); ++e) {
        size_t at = first;
        while (at < vox.size() && vox[at] != vx[e]) ++at;
        if (at == vox.size()) {
          vec.push_back(k);
          vox.push_back(vx[e]);
          val.insert(val.end(), 3, 0.0);
        }
        for (int c = 0; c < 3; ++c) val[3 * at + c] += pl[3 * e + c] * (e == 0 ? 1.0 : 0.1);
      }
    }
    require_distinct_entries(vec, vox);
    for (size_t e0 = 0; e0 < vec.size(); e0 += 80) {
      const int ne = (int)std::min<size_t>(80, vec.size() - e0);
      h2d(sm.vox, vox.data() + e0, ne * sizeof(long), s);
      h2d(sm.pol, val.data() + 3 * e0, 3 * ne * sizeof(double), s);
      h2d(sm.vox + 128, vec.data() + e0, ne * sizeof(long), s);
      launch_set_entries<T>(B, n3, g.nvox, ne, sm.vox + 128, sm.vox, sm.pol, s);
      BW_HIP(hipStreamSynchronize(s));
    }
  }
  // plus a small deterministic pseudo-random part (norm 1e-3 of the plane wave's),
  // so that the Krylov space is not confined to the reference plane waves: for a
  // homogeneous cell they are exact eigenvectors and the iteration would break
  // down after four steps
  // The seed is a function of the wave vector itself, so that a wave vector's start
  // (and result) does not depend on the batch it is solved in.
  for (int k = 0; k < nk; ++k)
    launch_add_hash<T>(B + (size_t)k * n3, n3, n3, 1, wave_vector_seed(k_list + 3 * k), 1e-3 / std::sqrt((double)n3),
                       s);
  apply_M_blk<T>(r, B, MF, nk, false, cnt, s);
  deflate_batch(B, MF, act);
  launch_dots<T>(B, MF, nk, n3, n3, sm.dots, r->ws_red, r->d_ctr + 64, s);
  std::vector<double2> bb(nk);
  BW_HIP(hipMemcpyAsync(bb.data(), sm.dots, nk * sizeof(double2), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < nk; ++k) sc[k] = 1.0 / std::sqrt(bb[k].x);
  upload_sc();
  launch_scale_copy<T>(B, n3, V, xk, scd, nk, n3, nullptr, s);
  if (!unit) launch_scale_copy<T>(MF, n3, MV, xk, scd, nk, n3, nullptr, s);

  std::vector<std::vector<double>> H(nk, std::vector<double>((size_t)m * m, 0.0));
  std::vector<double2> hh(hcount), hh2(hcount), cf((size_t)nk * ldc);
  std::vector<double> thv(m);
  std::vector<double2> Sm((size_t)m * m);
  int j0 = 0;
  int status = BW_OK;
  int cycles = 0;
  for (;;) {
    int nact = 0;
    for (int k = 0; k < nk; ++k) nact += act[k];
    if (nact == 0) break;
    upload_act();
    for (int j = j0; j < m; ++j) {
      // B_k = M v_j (zero for finished wave vectors), X = K^-1 B
      for (int k = 0; k < nk; ++k) sc[k] = act[k] ? 1.0 : 0.0;
      upload_sc();
      launch_scale_copy<T>(MV + (size_t)j * n3, xk, B, n3, scd, nk, n3, nullptr, s);
      // M v_j has no xi + k = 0 part for v_j M-orthogonal to the rigid translations;
      // drop the rounding left there, which the preconditioned iteration cannot reduce
      for (int k = 0; k < nk; ++k)
        if (act[k] && qt.null_index[k] >= 0) zero_voxel<T>(B + (size_t)k * n3, 1, g.nvox, qt.null_index[k], s);
      if constexpr (std::is_same<T, float>::value) {
        if (o.precond == BW_LEARNED) {
          // flexible PCG with the learned preconditioner (x0 = 0)
          BW_HIP(hipMemsetAsync(X, 0, (size_t)nk * n3 * sizeof(cplx<T>), s));
          const FpcgResult fr = fpcg_run(r, o.net, dq, qt, (const float2*)B, (float2*)X, nk,
                                         std::max(o.tol_lin, 1e-6), o.maxit_lin, s);
          cnt.pcg_iters += fr.total;
          cnt.kap += fr.total;
          for (int k = 0; k < nk; ++k) cnt.stalls += fr.fb[k] > 0;
        }
      }
      if (!(fp32 && o.precond == BW_LEARNED)) {
        PcgResult pr = pcg_run<T>(r, dq, qt, B, X, nk, fp32 ? std::max(o.tol_lin, 1e-6) : o.tol_lin, o.maxit_lin,
                                  true, s, false, false);
        cnt.pcg_iters += pr.total_iters;
        cnt.block_iters += pr.block_iters;
        cnt.kap += pr.k_applies;
      }
      // Full re-orthogonalization in the M inner product, twice, with the second
      // pass of each vector delayed by one step (classical Gram-Schmidt with delayed
      // re-orthogonalization): v_j was orthogonalized once when it was formed; one
      // pass of products over MV[0..j] with both v_j and X = OP v_j gives the
      // second-pass coefficients of v_j and the first-pass ones of X, and one
      // update pass over V[0..j-1] finishes v_j and orthogonalizes X against the
      // finished basis, X corrected for the change of v_j through the Lanczos
      // relation.  The basis is read twice per step instead of four times.
      launch_mdot2<T>(MV, xk, n3, j + 1, V + (size_t)j * n3, xk, X, n3, nk, n3, actd, hd, hd2, m + 1, r->ws_red, s);
      BW_HIP(hipMemcpyAsync(hh.data(), hd, hcount * sizeof(double2), hipMemcpyDeviceToHost, s));
      BW_HIP(hipMemcpyAsync(hh2.data(), hd2, hcount * sizeof(double2), hipMemcpyDeviceToHost, s));
      BW_HIP(hipStreamSynchronize(s));
      for (int k = 0; k < nk; ++k)
        if (act[k]) delayed_reorth_coefficients(H[k].data(), m, j, hh.data() + (size_t)k * (m + 1),
                                                hh2.data() + (size_t)k * (m + 1), cf.data() + (size_t)k * ldc);
      h2d(cfd, cf.data(), (size_t)nk * ldc * sizeof(double2), s);
      launch_mlincomb2<T>(V + (size_t)j * n3, xk, X, n3, V, xk, n3, j, cfd, ldc, nk, n3, actd, s);
      if (!unit) launch_mlincomb2<T>(MV + (size_t)j * n3, xk, nullptr, 0, MV, xk, n3, j, cfd, ldc, nk, n3, actd, s);
      if (unit) {
        // M' = I: M X is X, and the M-orthogonal projection off the rigid
        // translations (plane waves at xi + k = 0) zeroes that voxel
        for (int k = 0; k < nk; ++k)
          if (act[k] && qt.null_index[k] >= 0) zero_voxel<T>(X + (size_t)k * n3, 1, g.nvox, qt.null_index[k], s);
        launch_dots<T>(X, X, nk, n3, n3, sm.dots, r->ws_red, r->d_ctr + 64, s);
      } else {
        apply_M_blk<T>(r, X, MF, nk, false, cnt, s);
        deflate_batch(X, MF, act);
        launch_dots<T>(X, MF, nk, n3, n3, sm.dots, r->ws_red, r->d_ctr + 64, s);
      }
      BW_HIP(hipMemcpyAsync(bb.data(), sm.dots, nk * sizeof(double2), hipMemcpyDeviceToHost, s));
      BW_HIP(hipStreamSynchronize(s));
      for (int k = 0; k < nk; ++k) {
        if (!act[k]) {
          sc[k] = 0.0;
          continue;
        }
        beta[k] = std::sqrt(std::max(bb[k].x, 0.0));
        if (j + 1 < m) {
          H[k][(size_t)(j + 1) * m + j] = beta[k];
          H[k][(size_t)j * m + j + 1] = beta[k];
        }
        sc[k] = beta[k] > 0 ? 1.0 / beta[k] : 0.0;
      }
      upload_sc();
      launch_scale_copy<T>(X, n3, V + (size_t)(j + 1) * n3, xk, scd, nk, n3, actd, s);
      if (!unit) launch_scale_copy<T>(MF, n3, MV + (size_t)(j + 1) * n3, xk, scd, nk, n3, actd, s);
    }
    ++cycles;
    cnt.outer += 1;
    // projected eigenproblems of all active wave vectors in one launch
    std::vector<int> idx;
    for (int k = 0; k < nk; ++k)
      if (act[k]) idx.push_back(k);
    const int nb = (int)idx.size();
    std::vector<double> Hall((size_t)nb * m * m * 2, 0.0), thall((size_t)nb * m);
    std::vector<double2> Sall((size_t)nb * m * m);
    for (int b = 0; b < nb; ++b)
      for (size_t i = 0; i < (size_t)m * m; ++i) Hall[((size_t)b * m * m + i) * 2] = H[idx[b]][i];
    double2* Hd_dev = (double2*)w.v[9].get(Hall.size() * sizeof(double));
    double2* Sd_dev = (double2*)w.v[10].get((size_t)nb * m * m * sizeof(double2));
    double* th_dev = (double*)w.v[11].get((size_t)nb * m * sizeof(double) + (size_t)nb * sizeof(int) + 64);
    int* inf_dev = (int*)(th_dev + (size_t)nb * m);
    h2d(Hd_dev, Hall.data(), Hall.size() * sizeof(double), s);
    launch_small_eig_batched(Hd_dev, m, nb, th_dev, Sd_dev, inf_dev, s);
    BW_HIP(hipMemcpyAsync(thall.data(), th_dev, thall.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    BW_HIP(hipMemcpyAsync(Sall.data(), Sd_dev, Sall.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    BW_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b) {
      const int k = idx[b];
      std::copy(thall.begin() + (size_t)b * m, thall.begin() + (size_t)(b + 1) * m, thv.begin());
      std::copy(Sall.begin() + (size_t)b * m * m, Sall.begin() + (size_t)(b + 1) * m * m, Sm.begin());
      // the projected matrix is real symmetric, so are its eigenvectors: the Ritz
      // updates take real coefficients (complex ones if the solver left more than
      // rounding in the imaginary parts)
      double sm_im = 0;
      for (const double2& e : Sm) sm_im = std::max(sm_im, std::fabs(e.y));
      const bool rq = sm_im <= 1e-13;
      const int nw = nwk[k];
      bool conv = true;
      double worst = 0;
      for (int i = 0; i < nw; ++i) {
        const int c = m - 1 - i;  // largest theta first
        const double res = beta[k] * std::hypot(Sm[(size_t)(m - 1) * m + c].x, Sm[(size_t)(m - 1) * m + c].y);
        worst = std::max(worst, res / std::fabs(thv[c]));
        if (res > tolk[k] * std::fabs(thv[c])) conv = false;
      }
      if (verbose())
        fprintf(stderr, "[bw] lanczos k#%d cycle %d worst |beta s|/theta %.3e\n", kmap ? kmap[k] : kofs + k,
                cycles, worst);
      const bool last = cycles >= o.maxit_outer;
      if (conv || last) {
        // Ritz vectors of the wanted (and two more) values, then FP64 Rayleigh-Ritz and bounds
        std::vector<double2> Qs((size_t)m * qsel);
        for (int p = 0; p < m; ++p)
          for (int c = 0; c < qsel; ++c) Qs[(size_t)p * qsel + c] = Sm[(size_t)p * m + (m - 1 - c)];
        h2d(sm.Q, Qs.data(), Qs.size() * sizeof(double2), s);
        cplx<double>* U64 = ws<double>(r).vec(3, (size_t)qsel * n3);
        if (fp32) {
          launch_ritz<T>(V + (size_t)k * xk, m, sm.Q, qsel, TMP, qsel, n3, n3, s, rq);
          launch_convert<float, double>((const cplx<float>*)TMP, U64, (size_t)qsel * n3, s);
        } else {
          launch_ritz<T>(V + (size_t)k * xk, m, sm.Q, qsel, (cplx<T>*)U64, qsel, n3, n3, s, rq);
        }
        std::vector<double> k1((size_t)qsel * 3);
        for (int v = 0; v < qsel; ++v)
          for (int a = 0; a < 3; ++a) k1[3 * v + a] = k_list[3 * k + a];
        QTable qk = make_qtable(r, k1.data(), qsel);
        const double* dqk = upload_qtable(r, qk, r->ws_q3, s);
        std::vector<double> lam64, bnd;
        select_cell(kcell[k]);
        refine64<T>(r, dqk, qk, qt.null_index[k], qsel, nw, lam64, bnd, bound_target, 3, cnt, s);
        select_batch();
        const double wb = nw > 0 ? *std::max_element(bnd.begin(), bnd.end()) : 0.0;
        if (verbose()) fprintf(stderr, "[bw] lanczos k#%d FP64 bound %.3e\n", kmap ? kmap[k] : kofs + k, wb);
        const bool stalled = wb > 0.5 * best[k];  // the bound stopped improving (precision floor)
        best[k] = std::min(best[k], wb);
        if (wb <= bound_target || last || stalled) {
          if (wb > bound_target) status = BW_ENOTCONV;
          KOut ko;
          ko.n_want = nw;
          ko.jstar = qt.null_index[k];
          ko.lam.assign(lam64.begin(), lam64.begin() + nw);
          ko.bound = bnd;
          const int ik = kmap ? kmap[k] : kofs + k;
          int off = 0;
          if (ko.jstar >= 0) {
            for (int i = 0; i < 3; ++i) {
              omega[ik * nmodes + i] = 0.0;
              if (err) err[ik * nmodes + i] = 0.0;
            }
            off = 3;
          }
          for (int p = 0; p < nw; ++p) {
            omega[ik * nmodes + off + p] = std::sqrt(std::max(ko.lam[p], 0.0) * lscale);
            if (err) err[ik * nmodes + off + p] = ko.bound[p];
          }
          write_modes<T>(r, ko, nmodes, modes, ik, s);
          act[k] = 0;
          continue;
        }
        tolk[k] *= 0.1;  // tighten and keep iterating this wave vector
      }
      // thick restart: keep the kk leading Ritz vectors and the residual direction
      std::vector<double2> Qk((size_t)m * kk);
      for (int p = 0; p < m; ++p)
        for (int c = 0; c < kk; ++c) Qk[(size_t)p * kk + c] = Sm[(size_t)p * m + (m - 1 - c)];
      h2d(sm.Q, Qk.data(), Qk.size() * sizeof(double2), s);
      cplx<T>* Vk = V + (size_t)k * xk;
      cplx<T>* V2k = V2 + (size_t)k * xk;
      launch_ritz<T>(Vk, m, sm.Q, kk, V2k, kk, n3, n3, s, rq);
      BW_HIP(hipMemcpyAsync(V2k + (size_t)kk * n3, Vk + (size_t)m * n3, n3 * sizeof(cplx<T>),
                            hipMemcpyDeviceToDevice, s));
      if (!unit) {
        cplx<T>* MVk = MV + (size_t)k * xk;
        cplx<T>* MV2k = MV2 + (size_t)k * xk;
        launch_ritz<T>(MVk, m, sm.Q, kk, MV2k, kk, n3, n3, s, rq);
        BW_HIP(hipMemcpyAsync(MV2k + (size_t)kk * n3, MVk + (size_t)m * n3, n3 * sizeof(cplx<T>),
                              hipMemcpyDeviceToDevice, s));
      }
      std::fill(H[k].begin(), H[k].end(), 0.0);
      for (int c = 0; c < kk; ++c) {
        H[k][(size_t)c * m + c] = thv[m - 1 - c];
        // coupling of the kept Ritz vectors to the residual direction (the arrow
        // row of the restarted matrix), which the delayed re-orthogonalization of
        // that direction needs; its column is recomputed in the next step
        const double h = beta[k] * Sm[(size_t)(m - 1) * m + (m - 1 - c)].x;
        H[k][(size_t)kk * m + c] = h;
        H[k][(size_t)c * m + kk] = h;
      }
      BW_HIP(hipStreamSynchronize(s));
    }
    // the restarted wave vectors' bases are now in V2 (a finished one's basis is
    // no longer read)
    std::swap(V, V2);
    std::swap(MV, MV2);
    j0 = kk;
  }
  return status;
}

template <typename T>
static int lowest_modes_impl(bw_rve* r, const double* k_list, int nk, int nmodes, const EigOpts& o, double* omega,
                             double* err, void* modes, Counters& cnt, hipStream_t s) {
  const int q = o.block;
  bool have_start = false;
  std::vector<double> lam_prev;
  const double lscale = r->Cref / (r->rho_bar * r->ell * r->ell);
  int status = BW_OK;
  for (int ik = 0; ik < nk; ++ik) {
    if (!o.warm) have_start = false;
    KOut ko = subspace_k<T>(r, k_list + 3 * ik, nmodes, q, o, have_start, lam_prev, cnt, s);
    if (!ko.converged) status = BW_ENOTCONV;
    int off = 0;
    if (ko.jstar >= 0) {
      for (int i = 0; i < 3; ++i) {
        omega[ik * nmodes + i] = 0.0;
        if (err) err[ik * nmodes + i] = 0.0;
      }
      off = 3;
    }
    for (int p = 0; p < ko.n_want; ++p) {
      omega[ik * nmodes + off + p] = std::sqrt(std::max(ko.lam[p], 0.0) * lscale);
      if (err) err[ik * nmodes + off + p] = ko.bound[p];
    }
    write_modes<T>(r, ko, nmodes, modes, ik, s);
  }
  return status;
}

}  // namespace bw

using namespace bw;

extern "C" int bw_lowest_modes(bw_rve* r, const double* k_list, int32_t nk, int32_t nmodes, const bw_eig_opts* opts,
                               double* omega, double* err, void* modes, bw_stats* stats, void* stream) {
  try {
    BW_REQUIRE(r, BW_EINVAL, "null argument");
    BW_REQUIRE(nk >= 0, BW_EINVAL, "nk < 0");
    BW_REQUIRE(nmodes >= 1, BW_EINVAL, "nmodes must be >= 1");
    if (nk == 0) {
      if (stats) std::memset(stats, 0, sizeof(*stats));
      return BW_OK;
    }
    BW_REQUIRE(k_list && omega, BW_EINVAL, "null argument");
    BW_REQUIRE((long)nmodes <= 3 * r->g.nvox, BW_EINVAL, "more modes than degrees of freedom");
    EigOpts o{};
    if (opts) {
      o.method = opts->method;
      o.block = opts->block;
      o.ncv = opts->ncv;
      o.maxit_outer = opts->maxit_outer;
      o.maxit_lin = opts->maxit_lin;
      o.warm = opts->warm_start;
      o.tol_eig = opts->tol_eig;
      o.tol_lin = opts->tol_lin;
      o.tol_omega = opts->tol_omega;
      o.kbatch = opts->kbatch;
      o.precond = opts->precond;
      o.net = const_cast<bw_unet*>(opts->net);
      o.kgroups = opts->kgroups;
    } else {
      o.warm = 1;
    }
    BW_REQUIRE(o.method == BW_SUBSPACE || o.method == BW_LANCZOS, BW_EINVAL, "unknown method");
    BW_REQUIRE(o.precond == BW_PLAIN || o.precond == BW_LEARNED, BW_EINVAL, "unknown preconditioner");
    if (o.precond == BW_LEARNED) {
      BW_REQUIRE(o.net, BW_EINVAL, "BW_LEARNED needs a network");
      BW_REQUIRE(r->precision == BW_MIXED, BW_EINVAL, "the learned preconditioner works on BW_MIXED cells");
      BW_REQUIRE(o.method == BW_LANCZOS, BW_EUNSUPPORTED, "the learned preconditioner runs in the Lanczos solves");
      BW_REQUIRE(r->g.n0 % 4 == 0 && r->g.n1 % 4 == 0 && r->g.n2 % 4 == 0, BW_EUNSUPPORTED,
                 "the learned preconditioner needs grid sizes that are multiples of 4");
    }
    if (o.block <= 0) o.block = std::min(2 * nmodes, nmodes + 8);
    if (o.maxit_outer <= 0) o.maxit_outer = 200;
    if (o.maxit_lin <= 0) o.maxit_lin = 20000;
    if (o.tol_eig <= 0) o.tol_eig = 1e-10;
    if (o.tol_lin <= 0) o.tol_lin = r->precision == BW_FP64 ? 1e-10 : 1e-6;
    if (o.method == BW_SUBSPACE) {
      BW_REQUIRE(o.block > nmodes && o.block <= GRAM_QMAX, BW_EINVAL, "block must satisfy nmodes < block <= 32");
      BW_REQUIRE((long)o.block <= 3 * r->g.nvox, BW_EINVAL, "block larger than the number of degrees of freedom");
      // at a Gamma-like k the rigid translations leave 3 N - 3 degrees of freedom
      const QTable qt = make_qtable(r, k_list, nk);
      for (int k = 0; k < nk; ++k)
        BW_REQUIRE(qt.null_index[k] < 0 || (long)o.block <= 3 * r->g.nvox - 3, BW_EINVAL,
                   "block larger than the degrees of freedom at a Gamma-like wave vector (3 N - 3)");
    }
    hipStream_t s = (hipStream_t)stream;
    r->ws_red.get(16u << 20);
    r->ws_red2.get(16u << 20);
    Counters cnt;
    auto t0 = std::chrono::steady_clock::now();
    int st = BW_OK;
    if (o.method == BW_LANCZOS) {
      // wave vectors per batch: the bases within ~48 GB
      const int nwm = nmodes;
      const int m = o.ncv > 0 ? o.ncv : std::max(2 * nwm + 1, 20);
      const double vbytes = (double)r->g.nvox * 3 * (r->precision == BW_FP64 ? 16 : 8);
      // two bases per wave vector (restarts alternate between them), twice that
      // with their M-images when the density is not uniform
      const double nbases = r->rho_unit ? 2.0 : 4.0;
      int kb = (int)std::max(1.0, std::floor(48e9 / (vbytes * (nbases * (m + 1) + 3))));
      kb = std::min({kb, nk, 64});
      if (o.kbatch > 0) kb = std::min(kb, o.kbatch);
      // the wave vectors [ka, kz) on handle h and stream hs, in batches of kb
      auto run_range = [&](bw_rve* h, int ka, int kz, Counters& c, hipStream_t hs) {
        int stt = BW_OK;
        for (int k0 = ka; k0 < kz; k0 += kb) {
          const int nb = std::min(kb, kz - k0);
          const int s1 = h->precision == BW_FP64
                             ? lanczos_batch<double>(h, k_list + 3 * k0, nb, nmodes, o, omega, err, modes, k0, c, hs)
                             : lanczos_batch<float>(h, k_list + 3 * k0, nb, nmodes, o, omega, err, modes, k0, c, hs);
          if (s1 != BW_OK) stt = s1;
        }
        return stt;
      };
      const int ng = (r->ncell == 1 && !r->shared_tables && o.precond == BW_PLAIN)
                         ? std::min({std::max(o.kgroups, 1), nk, 8})
                         : 1;
      if (ng <= 1) {
        st = run_range(r, 0, nk, cnt, s);
      } else {
        // concurrent groups: one handle (the cell or a clone sharing its tables),
        // stream and host thread each.  Wave vector i goes to group i mod ng, so
        // that every group gets a share of each stretch of the path (neighbouring
        // wave vectors take similar numbers of restarts) and the groups end together.
        std::vector<std::vector<int>> ids(ng);
        std::vector<std::vector<double>> kls(ng);
        for (int i = 0; i < nk; ++i) {
          ids[i % ng].push_back(i);
          kls[i % ng].insert(kls[i % ng].end(), k_list + 3 * i, k_list + 3 * i + 3);
        }
        auto run_list = [&](bw_rve* hh, int gi, Counters& c, hipStream_t hs) {
          int stt = BW_OK;
          const int n = (int)ids[gi].size();
          for (int b0 = 0; b0 < n; b0 += kb) {
            const int nb = std::min(kb, n - b0);
            const double* kl = kls[gi].data() + 3 * b0;
            const int* km = ids[gi].data() + b0;
            const int s1 = hh->precision == BW_FP64
                               ? lanczos_batch<double>(hh, kl, nb, nmodes, o, omega, err, modes, 0, c, hs, km)
                               : lanczos_batch<float>(hh, kl, nb, nmodes, o, omega, err, modes, 0, c, hs, km);
            if (s1 != BW_OK) stt = s1;
          }
          return stt;
        };
        std::vector<bw_rve*> h(ng, r);
        for (int gi = 1; gi < ng; ++gi) {
          h[gi] = cell_clone(r, gi);
          h[gi]->ws_red.get(16u << 20);
          h[gi]->ws_red2.get(16u << 20);
        }
        BW_HIP(hipStreamSynchronize(s));
        std::vector<hipStream_t> gs(ng, nullptr);
        try {
          for (int gi = 0; gi < ng; ++gi) BW_HIP(hipStreamCreateWithFlags(&gs[gi], hipStreamNonBlocking));
        } catch (...) {
          for (auto x : gs)
            if (x) (void)hipStreamDestroy(x);
          throw;
        }
        std::vector<Counters> gc(ng);
        std::vector<int> code(ng, BW_OK);
        std::vector<std::string> msg(ng);
        std::vector<std::thread> th;
        th.reserve(ng);
        for (int gi = 0; gi < ng; ++gi)
          th.emplace_back([&, gi]() {
            try {
              BW_HIP(hipSetDevice(r->device));
              code[gi] = run_list(h[gi], gi, gc[gi], gs[gi]);
              BW_HIP(hipStreamSynchronize(gs[gi]));
            } catch (const Error& e) {
              code[gi] = e.code;
              msg[gi] = e.msg;
            } catch (const std::exception& e) {
              code[gi] = BW_EINVAL;
              msg[gi] = std::string("internal: ") + e.what();
            }
          });
        for (auto& t : th) t.join();
        for (auto x : gs) (void)hipStreamDestroy(x);
        for (int gi = 0; gi < ng; ++gi) {
          cnt.pcg_iters += gc[gi].pcg_iters;
          cnt.block_iters += gc[gi].block_iters;
          cnt.outer += gc[gi].outer;
          cnt.kap += gc[gi].kap;
          cnt.map += gc[gi].map;
          cnt.stalls += gc[gi].stalls;
          if (code[gi] < 0) throw Error{code[gi], msg[gi]};
          if (code[gi] != BW_OK) st = code[gi];
        }
      }
    } else {
      st = r->precision == BW_FP64 ? lowest_modes_impl<double>(r, k_list, nk, nmodes, o, omega, err, modes, cnt, s)
                                   : lowest_modes_impl<float>(r, k_list, nk, nmodes, o, omega, err, modes, cnt, s);
    }
    BW_HIP(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    if (stats) {
      stats->pcg_iterations = cnt.pcg_iters;
      stats->block_iterations = cnt.block_iters;
      stats->outer_iterations = cnt.outer;
      stats->k_applies = cnt.kap;
      stats->m_applies = cnt.map;
      stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    if (st == BW_ENOTCONV) set_error("bw_lowest_modes: some k hit maxit_outer; see the error bounds");
    if (st == BW_OK && cnt.stalls > 0) {
      set_error("bw_lowest_modes: the learned preconditioner stalled in " + std::to_string(cnt.stalls) +
                " inner solves, which finished with the plain preconditioner");
      st = BW_ESTALL;
    }
    return st;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal: ") + e.what());
    return BW_EINVAL;
  }
}

// Several cells at once.  Every cell runs the driver above on a stream of its own,
// from a host thread of its own, so that the kernels of small cells overlap on the
// GPU.  With opts->group_cells (Lanczos, no mode output), cells of one grid, cell
// edge and precision form a group instead: one handle whose batched launches carry
// the wave vectors of all its cells, each vector with its own cell's grain map and
// reference stiffness.  A cell's results are those of a separate call
// up to the rounding of the group's common scales (the same kernels, the same
// deterministic reductions; bit for bit for an ungrouped cell).
extern "C" int bw_lowest_modes_batched(bw_rve* const* rves, int32_t nrve, const double* const* k_lists,
                                       const int32_t* nks, int32_t nmodes, const bw_eig_opts* opts,
                                       double* const* omegas, double* const* errs, void* const* modes,
                                       bw_stats* stats, void* stream) {
  try {
    BW_REQUIRE(rves && k_lists && nks && omegas, BW_EINVAL, "null argument");
    BW_REQUIRE(nrve >= 0 && nrve <= 256, BW_EINVAL, "nrve out of range (0 .. 256)");
    for (int i = 0; i < nrve; ++i)
      BW_REQUIRE(rves[i] && (nks[i] == 0 || (k_lists[i] && omegas[i])), BW_EINVAL, "null cell argument");
    {
      // one host thread per cell: a handle is not thread-safe, so each may appear once
      std::vector<const bw_rve*> hs(rves, rves + nrve);
      std::sort(hs.begin(), hs.end());
      BW_REQUIRE(std::adjacent_find(hs.begin(), hs.end()) == hs.end(), BW_EINVAL,
                 "the same cell handle appears twice in the batch");
    }
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t cs = (hipStream_t)stream;
    // work already queued on the caller's stream precedes the batch
    BW_HIP(hipStreamSynchronize(cs));
    // units of work: groups of cells of one grid, cell edge and precision, and single cells
    const bool may_group = opts && opts->method == BW_LANCZOS && !modes && opts->group_cells &&
                           opts->precond != BW_LEARNED;
    auto same_kind = [](const bw_rve* a, const bw_rve* b) {
      return a->ncell == 1 && b->ncell == 1 && a->g.n0 == b->g.n0 && a->g.n1 == b->g.n1 && a->g.n2 == b->g.n2 &&
             a->precision == b->precision && a->device == b->device && a->L[0] == b->L[0] && a->L[1] == b->L[1] &&
             a->L[2] == b->L[2];
    };
    std::vector<std::vector<int>> units;
    {
      std::vector<char> used(nrve, 0);
      for (int i = 0; i < nrve; ++i) {
        if (used[i]) continue;
        std::vector<int> u = {i};
        used[i] = 1;
        if (may_group && nks[i] > 0)
          for (int j = i + 1; j < nrve && (int)u.size() < CELLS_MAX; ++j)
            if (!used[j] && nks[j] > 0 && same_kind(rves[i], rves[j])) {
              u.push_back(j);
              used[j] = 1;
            }
        units.push_back(u);
      }
    }
    const int nu = (int)units.size();
    int cur = 0;
    BW_HIP(hipGetDevice(&cur));
    // group handles (built here, not on the worker threads: allocation is serialized
    // with graph captures) and their concatenated wave-vector lists
    std::vector<bw_rve*> uh(nu, nullptr);
    std::vector<std::vector<double>> ukl(nu), uom(nu), uer(nu);
    try {
      for (int u = 0; u < nu; ++u) {
        const std::vector<int>& c = units[u];
        if (c.size() == 1) {
          uh[u] = rves[c[0]];
          continue;
        }
        BW_HIP(hipSetDevice(rves[c[0]]->device));
        std::vector<bw_rve*> cells;
        for (int i : c) cells.push_back(rves[i]);
        bw_rve* gr = cell_group(cells.data(), (int)cells.size());
        gr->kcell_bounds.assign(1, 0);
        for (int i : c) {
          ukl[u].insert(ukl[u].end(), k_lists[i], k_lists[i] + 3 * (size_t)nks[i]);
          gr->kcell_bounds.push_back(gr->kcell_bounds.back() + nks[i]);
        }
        const size_t nkt = (size_t)gr->kcell_bounds.back();
        uom[u].assign(nkt * nmodes, 0.0);
        uer[u].assign(nkt * nmodes, 0.0);
        uh[u] = gr;
      }
      BW_HIP(hipSetDevice(cur));
    } catch (...) {
      (void)hipSetDevice(cur);
      throw;
    }
    std::vector<hipStream_t> st(nu, nullptr);
    std::vector<int> code(nu, BW_OK);
    std::vector<std::string> msg(nu);
    std::vector<bw_stats> one(nu);
    try {
      for (int u = 0; u < nu; ++u) {
        BW_HIP(hipSetDevice(uh[u]->device));
        BW_HIP(hipStreamCreateWithFlags(&st[u], hipStreamNonBlocking));
      }
      BW_HIP(hipSetDevice(cur));
    } catch (...) {
      for (auto x : st)
        if (x) (void)hipStreamDestroy(x);
      (void)hipSetDevice(cur);
      throw;
    }
    std::vector<std::thread> th;
    th.reserve(nu);
    for (int u = 0; u < nu; ++u)
      th.emplace_back([&, u]() {
        if (hipSetDevice(uh[u]->device) != hipSuccess) {
          code[u] = BW_EHIP;
          msg[u] = "hipSetDevice failed";
          return;
        }
        std::memset(&one[u], 0, sizeof(bw_stats));
        const std::vector<int>& c = units[u];
        if (c.size() == 1) {
          const int i = c[0];
          code[u] = bw_lowest_modes(rves[i], k_lists[i], nks[i], nmodes, opts, omegas[i], errs ? errs[i] : nullptr,
                                    modes ? modes[i] : nullptr, &one[u], st[u]);
        } else {
          code[u] = bw_lowest_modes(uh[u], ukl[u].data(), (int)(ukl[u].size() / 3), nmodes, opts, uom[u].data(),
                                    uer[u].data(), nullptr, &one[u], st[u]);
        }
        if (code[u] != BW_OK) msg[u] = bw_last_error();
      });
    for (auto& t : th) t.join();
    for (auto x : st) (void)hipStreamDestroy(x);
    // the groups' rows back to their cells
    for (int u = 0; u < nu; ++u) {
      const std::vector<int>& c = units[u];
      if (c.size() == 1) continue;
      size_t row = 0;
      for (int i : c) {
        const size_t n = (size_t)nks[i] * nmodes;
        std::copy(uom[u].begin() + row, uom[u].begin() + row + n, omegas[i]);
        if (errs && errs[i]) std::copy(uer[u].begin() + row, uer[u].begin() + row + n, errs[i]);
        row += n;
      }
    }
    int status = BW_OK;
    std::string first;
    for (int u = 0; u < nu; ++u) {
      if (code[u] < 0 && (status >= 0 || code[u] < status)) status = code[u];
      if (code[u] == BW_ENOTCONV && status == BW_OK) status = BW_ENOTCONV;
      if (code[u] != BW_OK && first.empty()) {
        std::string who = "cell";
        for (int i : units[u]) who += " " + std::to_string(i);
        first = who + ": " + msg[u];
      }
    }
    if (stats) {
      std::memset(stats, 0, sizeof(bw_stats));
      for (auto& o : one) {
        stats->pcg_iterations += o.pcg_iterations;
        stats->block_iterations += o.block_iterations;
        stats->outer_iterations += o.outer_iterations;
        stats->k_applies += o.k_applies;
        stats->m_applies += o.m_applies;
      }
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status != BW_OK) set_error(first);
    return status;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal: ") + e.what());
    return BW_EINVAL;
  }
}
