// Dispersion post-processing: slopes of the branches (group velocity, Sec. 5.1
// eq. c_group) and long-wave speeds of the three acoustic branches.
//
// Slopes.  K(k) depends on k only through the shifted frequencies q = xi + k of
// the strain and the divergence (Sec. 3.2 eq. hatA), each linear in q, so K is a
// quadratic polynomial in k and U^H K(k + h d) U = A + h D + h^2 Q exactly:
//   D = U^H (dK/ds) U = U^H [K(k + h d) - K(k - h d)] U / (2h)
// for any step h.  The slopes d omega / ds are the eigenvalues of the pencil
// (D, U^H M U) on each cluster of equal omega divided by 2 omega (first-order
// perturbation of omega^2 = U^H K U / U^H M U; M does not depend on k).  Two K
// applies and one M apply of the mode block in FP64, three Gram products, and
// one small generalized eigenproblem per cluster.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "bw_block.h"

using namespace bw;

namespace {

// A step h such that neither k + h d nor k - h d lies within 1e-6 (in units of
// 2 pi / L) of a reciprocal-lattice vector, where wave vectors are snapped.
double pick_step(const bw_rve* r, const double* k, const double* d) {
  const double Lmax = std::max({r->L[0], r->L[1], r->L[2]});
  double h = M_PI / (4.0 * Lmax);
  for (int t = 0; t < 32; ++t, h *= 0.77) {
    bool ok = true;
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      bool near = true;
      for (int a = 0; a < 3; ++a) {
        const double kap = (k[a] + sgn * h * d[a]) * r->L[a] / (2.0 * M_PI);
        if (std::fabs(kap - std::nearbyint(kap)) > 1e-6) near = false;
      }
      if (near) ok = false;
    }
    if (ok) break;
  }
  return h;
}

double unit_direction(const double* dir, double* d) {
  const double n = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  BW_REQUIRE(n > 0 && std::isfinite(n), BW_EINVAL, "direction must be a nonzero finite vector");
  for (int a = 0; a < 3; ++a) d[a] = dir[a] / n;
  return n;
}

}  // namespace

extern "C" int bw_group_velocity(bw_rve* r, const double k[3], const double dir[3], int32_t nmodes,
                                 const void* modes, const double* omega_host, double cluster_tol,
                                 double* slopes_host, void* stream) {
  try {
    BW_REQUIRE(r && k && dir && modes && omega_host && slopes_host, BW_EINVAL, "null argument");
    BW_REQUIRE(nmodes >= 1 && nmodes <= GRAM_QMAX, BW_EINVAL, "nmodes must be in 1 .. 32");
    BW_REQUIRE(cluster_tol >= 0 && cluster_tol < 1, BW_EINVAL, "cluster_tol must be in [0, 1)");
    for (int a = 0; a < 3; ++a) BW_REQUIRE(std::isfinite(k[a]), BW_EINVAL, "non-finite wave vector");
    double d[3];
    unit_direction(dir, d);
    for (int p = 0; p < nmodes; ++p) {
      BW_REQUIRE(std::isfinite(omega_host[p]) && omega_host[p] >= 0, BW_EINVAL, "omega must be finite and >= 0");
      BW_REQUIRE(p == 0 || omega_host[p] >= omega_host[p - 1], BW_EINVAL, "omega must be ascending");
    }
    hipStream_t s = (hipStream_t)stream;
    const int nm = nmodes;
    const long n3 = 3 * r->g.nvox;
    Workspace<double>& w = ws<double>(r);
    const cplx<double>* U;
    if (r->precision == BW_FP64) {
      U = (const cplx<double>*)modes;
    } else {
      cplx<double>* U64 = w.vec(13, (size_t)nm * n3);
      launch_convert<float, double>((const cplx<float>*)modes, U64, (size_t)nm * n3, s);
      U = U64;
    }
    cplx<double>* Y = w.vec(14, (size_t)nm * n3);
    cplx<double>* W = w.work((size_t)nm * 6 * r->g.nvox);
    const size_t nq = (size_t)nm * nm;
    double2* G = (double2*)r->ws_misc.get(3 * nq * sizeof(double2));
    const double h = pick_step(r, k, d);
    std::vector<QTable> qts;
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      std::vector<double> kk((size_t)3 * nm);
      for (int v = 0; v < nm; ++v)
        for (int a = 0; a < 3; ++a) kk[3 * v + a] = k[a] + sgn * h * d[a];
      qts.push_back(make_qtable(r, kk.data(), nm));
      const double* dq = upload_qtable(r, qts.back(), r->ws_q3, s);
      launch_apply_K<double>(r, dq, U, Y, nm, K_scale(r), W, s);
      launch_gram<double>(U, nm, Y, nm, n3, n3, G + (sgn > 0 ? 0 : nq), r->ws_red, r->d_ctr, s);
    }
    launch_apply_M<double>(r, U, Y, nm, M_scale(r), W, s);
    launch_gram<double>(U, nm, Y, nm, n3, n3, G + 2 * nq, r->ws_red, r->d_ctr, s);
    std::vector<double2> gh(3 * nq);
    BW_HIP(hipMemcpyAsync(gh.data(), G, 3 * nq * sizeof(double2), hipMemcpyDeviceToHost, s));
    BW_HIP(hipStreamSynchronize(s));
    // Hermitian parts: D = (G+ - G-) / 2h, B = U^H M U
    std::vector<double2> D(nq), B(nq);
    for (int i = 0; i < nm; ++i)
      for (int j = 0; j < nm; ++j) {
        const size_t ij = (size_t)i * nm + j, ji = (size_t)j * nm + i;
        const double dr = (gh[ij].x - gh[nq + ij].x) / (2 * h), di = (gh[ij].y - gh[nq + ij].y) / (2 * h);
        const double dr2 = (gh[ji].x - gh[nq + ji].x) / (2 * h), di2 = (gh[ji].y - gh[nq + ji].y) / (2 * h);
        D[ij] = double2{0.5 * (dr + dr2), 0.5 * (di - di2)};
        B[ij] = double2{0.5 * (gh[2 * nq + ij].x + gh[2 * nq + ji].x), 0.5 * (gh[2 * nq + ij].y - gh[2 * nq + ji].y)};
      }
    // clusters of equal omega (relative gap <= cluster_tol)
    std::vector<std::vector<int>> cl(1, std::vector<int>{0});
    for (int p = 1; p < nm; ++p) {
      if (omega_host[p] - omega_host[p - 1] <= cluster_tol * std::max(omega_host[p], 1e-300))
        cl.back().push_back(p);
      else
        cl.push_back(std::vector<int>{p});
    }
    for (auto& c : cl) {
      double wc = 0;
      for (int p : c) wc += omega_host[p];
      wc /= (double)c.size();
      if (wc == 0.0) {
        for (int p : c) slopes_host[p] = 0.0;
        continue;
      }
      const int q = (int)c.size();
      if (q == 1) {
        const size_t pp = (size_t)c[0] * nm + c[0];
        slopes_host[c[0]] = D[pp].x / B[pp].x / (2 * wc);
        continue;
      }
      BW_REQUIRE(q <= GEIG_QMAX, BW_EINVAL, "cluster too large");
      std::vector<double2> Dc((size_t)q * q), Bc((size_t)q * q);
      for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
          Dc[(size_t)i * q + j] = D[(size_t)c[i] * nm + c[j]];
          Bc[(size_t)i * q + j] = B[(size_t)c[i] * nm + c[j]];
        }
      char* sb = (char*)r->ws_misc.get(3 * nq * sizeof(double2) + 3 * (size_t)q * q * sizeof(double2) +
                                       q * sizeof(double) + 64);
      G = (double2*)sb;   // the buffer may have moved; G is not read again
      double2* dK = (double2*)(sb + 3 * nq * sizeof(double2));
      double2* dM = dK + (size_t)q * q;
      double2* dQ = dM + (size_t)q * q;
      double* dl = (double*)(dQ + (size_t)q * q);
      int* dinfo = (int*)(dl + q);
      BW_HIP(hipMemcpyAsync(dK, Dc.data(), Dc.size() * sizeof(double2), hipMemcpyHostToDevice, s));
      BW_HIP(hipMemcpyAsync(dM, Bc.data(), Bc.size() * sizeof(double2), hipMemcpyHostToDevice, s));
      launch_small_geig(dK, dM, q, dl, dQ, dinfo, s);
      std::vector<double> lam(q);
      int info = 0;
      BW_HIP(hipMemcpyAsync(lam.data(), dl, q * sizeof(double), hipMemcpyDeviceToHost, s));
      BW_HIP(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
      BW_HIP(hipStreamSynchronize(s));
      BW_REQUIRE(info == 0, BW_EINVAL, "U^H M U of a cluster is not positive definite (modes not independent)");
      for (int i = 0; i < q; ++i) slopes_host[c[i]] = lam[i] / (2 * wc);
    }
    return BW_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal: ") + e.what());
    return BW_EINVAL;
  }
}

// Long-wave speeds: omega_i / |k| of the three lowest branches at k = h d and
// 2h d (one bw_lowest_modes call, subspace iteration: a block method resolves the
// degenerate transverse pairs of symmetric cells, which a single-vector Krylov
// method finds only once); omega^2 is even and analytic in k,
// so omega / |k| = c + O(k^2) and the extrapolation (4 c(h) - c(2h)) / 3 leaves
// O(h^4).  The limit is the speed of the equivalent homogeneous medium (Sec.
// 5.1: d omega / dk tends to it for k -> 0).
extern "C" int bw_long_wave_speeds(bw_rve* r, const double dir[3], double h_frac, double tol_omega, double* c_host,
                                   void* stream) {
  try {
    BW_REQUIRE(r && dir && c_host, BW_EINVAL, "null argument");
    BW_REQUIRE(h_frac > 0 && h_frac <= 0.25, BW_EINVAL, "h_frac must be in (0, 0.25]");
    BW_REQUIRE(tol_omega >= 0 && tol_omega < 1e-2, BW_EINVAL, "tol_omega must be in [0, 1e-2)");
    BW_REQUIRE(3 * r->g.nvox >= 4, BW_EINVAL, "cell too small");
    double d[3];
    unit_direction(dir, d);
    const double Lmax = std::max({r->L[0], r->L[1], r->L[2]});
    const double h = h_frac * M_PI / Lmax;
    double ks[6];
    for (int a = 0; a < 3; ++a) {
      ks[a] = h * d[a];
      ks[3 + a] = 2 * h * d[a];
    }
    bw_eig_opts o;
    std::memset(&o, 0, sizeof(o));
    o.method = BW_SUBSPACE;
    o.warm_start = 1;
    o.tol_omega = tol_omega > 0 ? tol_omega : (r->precision == BW_FP64 ? 1e-10 : 1e-8);
    o.tol_lin = r->precision == BW_FP64 ? std::min(1e-10, 0.1 * o.tol_omega) : 1e-6;
    double om[6];
    const int code = bw_lowest_modes(r, ks, 2, 3, &o, om, nullptr, nullptr, nullptr, stream);
    if (code < 0) return code;
    std::sort(om, om + 3);
    std::sort(om + 3, om + 6);
    for (int i = 0; i < 3; ++i) c_host[i] = (4.0 * om[i] / h - om[3 + i] / (2.0 * h)) / 3.0;
    return code;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal: ") + e.what());
    return BW_EINVAL;
  }
}
