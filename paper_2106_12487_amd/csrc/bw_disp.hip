// Dispersion post-processing: slopes of the branches (group velocity, Sec. 5.1
// eq. c_group), long-wave speeds of the three acoustic branches, the static
// homogenization they tend to (effective stiffness), and real-space mode fields
// with strain maps (Sec. 5.2, eq. rotate_eigenvector).
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
#include <limits>
#include <string>
#include <vector>

#include "bw_block.h"
#include "bw_ops_impl.h"

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
      h2d(dK, Dc.data(), Dc.size() * sizeof(double2), s);
      h2d(dM, Bc.data(), Bc.size() * sizeof(double2), s);
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
    // k = h d, -h d, 2h d, -2h d: the mean of omega over +-k is even in k (on an even
    // grid the frequency set alone is not, the Nyquist label -N/2 having no +N/2)
    double ks[12];
    for (int a = 0; a < 3; ++a) {
      ks[a] = h * d[a];
      ks[3 + a] = -h * d[a];
      ks[6 + a] = 2 * h * d[a];
      ks[9 + a] = -2 * h * d[a];
    }
    bw_eig_opts o;
    std::memset(&o, 0, sizeof(o));
    o.method = BW_SUBSPACE;
    o.warm_start = 1;
    o.tol_omega = tol_omega > 0 ? tol_omega : (r->precision == BW_FP64 ? 1e-10 : 1e-8);
    o.tol_lin = r->precision == BW_FP64 ? std::min(1e-10, 0.1 * o.tol_omega) : 1e-6;
    double om[12];
    const int code = bw_lowest_modes(r, ks, 4, 3, &o, om, nullptr, nullptr, nullptr, stream);
    if (code < 0) return code;
    for (int j = 0; j < 4; ++j) std::sort(om + 3 * j, om + 3 * j + 3);
    for (int i = 0; i < 3; ++i) {
      const double c1 = (om[i] + om[3 + i]) / (2.0 * h), c2 = (om[6 + i] + om[9 + i]) / (4.0 * h);
      c_host[i] = (4.0 * c1 - c2) / 3.0;
    }
    return code;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal: ") + e.what());
    return BW_EINVAL;
  }
}

// ---------------------------------------------------------------------------
// Real-space mode fields (Sec. 5.2, eigenvectors, eq. rotate_eigenvector):
// U(x) = e^{-i phi} F^-1(U^) with phi = arg(sum_x U . U) / 2, the phase that makes
// the field as close to real as it can be (for a field of common phase, that
// phase, up to pi); strain eps(x) = e^{-i phi} F^-1[i B(xi + k) U^] (Voigt,
// engineering shear), the strain of the Bloch wave U(x) e^{i k.x} divided by its
// phase factor e^{i k.x}.
// ---------------------------------------------------------------------------
namespace {

// unnormalized 3D FFT (INV: inverse) of nv fields of nc components, in place
template <typename T, bool INV> void fft3_nc(const bw_rve* r, cplx<T>* X, int nv, int nc, hipStream_t s) {
  const Geom& g = r->g;
  const long rows = (long)nc * g.n0 * g.n1;
  with_n(g.n2, [&](auto N2) {
    constexpr int n2c = decltype(N2)::value;
    RowTile rt = row_tile<T>(n2c, rows);
    hipLaunchKernelGGL((k_row_plain<T, n2c, INV>), dim3(nv * rt.tpv), dim3(NT), 0, s, (const cplx<T>*)X, X, rt,
                       (int)rows, twiddles<T>(r, 2), (const int*)nullptr);
  });
  if (g.n1 > 1)
    with_n(g.n1, [&](auto N1) {
      ColTile ct = axis1_tile<T>(N1, g.n2, (long)nc * g.n0 * g.n2);
      hipLaunchKernelGGL((k_axis1<T, decltype(N1)::value, INV>), dim3(nv * ct.tpv), dim3(NT), 0, s, X, g.n2,
                         (long)nc * g.nvox, ct, twiddles<T>(r, 1), (const int*)nullptr);
    });
  if (g.n0 > 1) {
    const int n12 = g.n1 * g.n2;
    with_n(g.n0, [&](auto N0) {
      ColTile ct = axis1_tile<T>(N0, n12, (long)nc * n12);
      hipLaunchKernelGGL((k_axis1<T, decltype(N0)::value, INV>), dim3(nv * ct.tpv), dim3(NT), 0, s, X, n12,
                         (long)nc * g.nvox, ct, twiddles<T>(r, 0), (const int*)nullptr);
    });
  }
}

// E = i B(q) U per Fourier voxel; q = qscale * table (the table of one wave vector)
template <typename T>
__global__ void k_strain_hat(const cplx<T>* __restrict__ U, const double* __restrict__ qtab, cplx<T>* __restrict__ E,
                             int n0, int n1, int n2, long nvox, int nv, double qscale) {
  const long total = (long)nv * nvox;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long v = e / nvox, x = e - v * nvox;
    const int i2 = (int)(x % n2), i1 = (int)((x / n2) % n1), i0 = (int)(x / ((long)n1 * n2));
    const double qa = qscale * qtab[i0], qb = qscale * qtab[n0 + i1], qc = qscale * qtab[n0 + n1 + i2];
    double ur[3], ui[3];
    for (int c = 0; c < 3; ++c) {
      const cplx<T> u = U[((size_t)v * 3 + c) * nvox + x];
      ur[c] = (double)u.x;
      ui[c] = (double)u.y;
    }
    // Voigt strain [q1 U1, q2 U2, q3 U3, q3 U2 + q2 U3, q3 U1 + q1 U3, q2 U1 + q1 U2], times i
    const double sr[6] = {qa * ur[0], qb * ur[1], qc * ur[2], qc * ur[1] + qb * ur[2], qc * ur[0] + qa * ur[2],
                          qb * ur[0] + qa * ur[1]};
    const double si[6] = {qa * ui[0], qb * ui[1], qc * ui[2], qc * ui[1] + qb * ui[2], qc * ui[0] + qa * ui[2],
                          qb * ui[0] + qa * ui[1]};
    for (int c = 0; c < 6; ++c) {
      cplx<T> o;
      o.x = (T)(-si[c]);
      o.y = (T)sr[c];
      E[((size_t)v * 6 + c) * nvox + x] = o;
    }
  }
}

// per-block partial sums of (Re, Im) of sum U . U over nc components, bpv blocks per field
template <typename T>
__global__ void k_square_sum(const cplx<T>* __restrict__ X, long n, int bpv, double* __restrict__ part) {
  __shared__ double sh[2][256];
  const int v = blockIdx.x / bpv, b = blockIdx.x - v * bpv;
  double re = 0, im = 0;
  for (long e = (long)b * blockDim.x + threadIdx.x; e < n; e += (long)bpv * blockDim.x) {
    const cplx<T> u = X[(size_t)v * n + e];
    re += (double)u.x * u.x - (double)u.y * u.y;
    im += 2.0 * (double)u.x * u.y;
  }
  sh[0][threadIdx.x] = re;
  sh[1][threadIdx.x] = im;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * ((size_t)v * bpv + b)] = sh[0][0];
    part[2 * ((size_t)v * bpv + b) + 1] = sh[1][0];
  }
}

// X_v *= c_v (complex, device) over n elements per field
template <typename T>
__global__ void k_scale_fields(cplx<T>* X, long n, int nv, const double2* __restrict__ c) {
  const long total = (long)nv * n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const double2 f = c[e / n];
    const cplx<T> u = X[e];
    cplx<T> o;
    o.x = (T)(f.x * (double)u.x - f.y * (double)u.y);
    o.y = (T)(f.x * (double)u.y + f.y * (double)u.x);
    X[e] = o;
  }
}

unsigned grid_of(long total) {
  long b = (total + 255) / 256;
  return (unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

template <typename T>
void mode_fields(bw_rve* r, const double* k, int nm, const cplx<T>* Uh, cplx<T>* u, cplx<T>* eps, double* phase,
                 hipStream_t s) {
  const Geom& g = r->g;
  const long n3 = 3 * g.nvox;
  BW_HIP(hipMemcpyAsync(u, Uh, (size_t)nm * n3 * sizeof(cplx<T>), hipMemcpyDeviceToDevice, s));
  fft3_nc<T, true>(r, u, nm, 3, s);
  const int bpv = 64;
  double* part = (double*)r->ws_misc.get((size_t)nm * bpv * 2 * sizeof(double) + (size_t)nm * sizeof(double2));
  double2* coef = (double2*)(part + (size_t)nm * bpv * 2);
  hipLaunchKernelGGL((k_square_sum<T>), dim3((unsigned)(nm * bpv)), dim3(256), 0, s, (const cplx<T>*)u, n3, bpv,
                     part);
  std::vector<double> ph((size_t)nm * bpv * 2);
  BW_HIP(hipMemcpyAsync(ph.data(), part, ph.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  std::vector<double2> cf(nm);
  for (int v = 0; v < nm; ++v) {
    double re = 0, im = 0;
    for (int b = 0; b < bpv; ++b) {
      re += ph[2 * ((size_t)v * bpv + b)];
      im += ph[2 * ((size_t)v * bpv + b) + 1];
    }
    const double phi = 0.5 * std::atan2(im, re);
    if (phase) phase[v] = phi;
    // e^{-i phi} / N (the inverse transform above is unnormalized)
    cf[v] = double2{std::cos(phi) / (double)g.nvox, -std::sin(phi) / (double)g.nvox};
  }
  h2d(coef, cf.data(), nm * sizeof(double2), s);
  hipLaunchKernelGGL((k_scale_fields<T>), dim3(grid_of((long)nm * n3)), dim3(256), 0, s, u, n3, nm,
                     (const double2*)coef);
  if (eps) {
    QTable qt = make_qtable(r, k, 1);
    const double* dq = upload_qtable(r, qt, r->ws_q3, s);
    hipLaunchKernelGGL((k_strain_hat<T>), dim3(grid_of((long)nm * g.nvox)), dim3(256), 0, s, Uh, dq, eps, g.n0, g.n1,
                       g.n2, g.nvox, nm, 1.0 / r->ell);
    fft3_nc<T, true>(r, eps, nm, 6, s);
    hipLaunchKernelGGL((k_scale_fields<T>), dim3(grid_of((long)nm * 6 * g.nvox)), dim3(256), 0, s, eps,
                       6 * g.nvox, nm, (const double2*)coef);
  }
  BW_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Static homogenization, the long-wave limit of the Bloch problem (Sec. 5.1).
// For each unit macro strain E_j (Voigt, engineering shear) the periodic
// fluctuation u solves K(0) u^ = i B(xi)^H F[C(x) E_j] (equilibrium of
// C (E_j + eps(u)) with eps(u) = F^-1[i B(xi) u^]; PCG, Algorithm "InvA"), and
// column j of C_eff is the volume mean of C(x) (E_j + eps(u)).  In the cell's
// scaled units (C' = C / Cref, q' = q ell) the factors ell cancel:
// u'^ = K'(0)^-1 b' with b' = i B(xi')^H F[C' E_j], eps = F^-1[i B(xi') u'^].
// On an even grid the Nyquist label -n/2 has no partner +n/2, the fluctuation
// is not real, and the real part of the mean stress is taken.
// ---------------------------------------------------------------------------
// S[j][c][x] = C'(x)_{c j}: the stress of E_j, real, all six j
template <typename T>
__global__ void k_unit_stress(const uint16_t* __restrict__ gmap, const T* __restrict__ C, cplx<T>* __restrict__ S,
                              long nvox) {
  for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < nvox; x += (long)gridDim.x * blockDim.x) {
    const int g = gmap[x];
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        cplx<T> o;
        o.x = C[g * 21 + vidx(c, j)];
        o.y = 0;
        S[((size_t)j * 6 + c) * nvox + x] = o;
      }
  }
}

// B = i B(q)^H S per Fourier voxel (q = qscale * table of one wave vector):
// out_i = i sum_m q_m S_{i m} with the Voigt stress S
template <typename T>
__global__ void k_div_hat(const cplx<T>* __restrict__ S, const double* __restrict__ qtab, cplx<T>* __restrict__ B,
                          int n0, int n1, int n2, long nvox, int nv, double qscale) {
  const long total = (long)nv * nvox;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long v = e / nvox, x = e - v * nvox;
    const int i2 = (int)(x % n2), i1 = (int)((x / n2) % n1), i0 = (int)(x / ((long)n1 * n2));
    const double qa = qscale * qtab[i0], qb = qscale * qtab[n0 + i1], qc = qscale * qtab[n0 + n1 + i2];
    double sr[6], si[6];
    for (int c = 0; c < 6; ++c) {
      const cplx<T> u = S[((size_t)v * 6 + c) * nvox + x];
      sr[c] = (double)u.x;
      si[c] = (double)u.y;
    }
    const double rr[3] = {qa * sr[0] + qb * sr[5] + qc * sr[4], qa * sr[5] + qb * sr[1] + qc * sr[3],
                          qa * sr[4] + qb * sr[3] + qc * sr[2]};
    const double ri[3] = {qa * si[0] + qb * si[5] + qc * si[4], qa * si[5] + qb * si[1] + qc * si[3],
                          qa * si[4] + qb * si[3] + qc * si[2]};
    for (int c = 0; c < 3; ++c) {
      cplx<T> o;
      o.x = (T)(-ri[c]);
      o.y = (T)rr[c];
      B[((size_t)v * 3 + c) * nvox + x] = o;
    }
  }
}

// per-block partial sums over voxels of C'(x) (E_j + Re(eps) inv_n), eps the
// unnormalized inverse transform of the strain of field j; bpv blocks per j
template <typename T>
__global__ __launch_bounds__(256) void k_mean_stress(const uint16_t* __restrict__ gmap, const T* __restrict__ C,
                                                     const cplx<T>* __restrict__ Eps, long nvox, double inv_n, int bpv,
                                                     double* __restrict__ part) {
  __shared__ double sh[6][256];
  const int j = blockIdx.x / bpv, b = blockIdx.x - j * bpv;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long x = (long)b * 256 + threadIdx.x; x < nvox; x += (long)bpv * 256) {
    const int g = gmap[x];
    double e[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) e[c] = (c == j ? 1.0 : 0.0) + (double)Eps[((size_t)j * 6 + c) * nvox + x].x * inv_n;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double sa = 0;
#pragma unroll
      for (int c = 0; c < 6; ++c) sa += (double)C[g * 21 + vidx(a, c)] * e[c];
      acc[a] += sa;
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) sh[a][threadIdx.x] = acc[a];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int a = 0; a < 6; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int a = 0; a < 6; ++a) part[((size_t)j * bpv + b) * 6 + a] = sh[a][0];
}

// per-block partial sums of |X|^2 over n elements per field, bpv blocks per field
template <typename T>
__global__ __launch_bounds__(256) void k_norm2(const cplx<T>* __restrict__ X, long n, int bpv,
                                               double* __restrict__ part) {
  __shared__ double sh[256];
  const int v = blockIdx.x / bpv, b = blockIdx.x - v * bpv;
  double a = 0;
  for (long e = (long)b * 256 + threadIdx.x; e < n; e += (long)bpv * 256) {
    const cplx<T> u = X[(size_t)v * n + e];
    a += (double)u.x * u.x + (double)u.y * u.y;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)v * bpv + b] = sh[0];
}

template <typename T>
std::vector<double> field_norms2(const cplx<T>* X, int nv, long n, double* part, int bpv, hipStream_t s) {
  hipLaunchKernelGGL((k_norm2<T>), dim3((unsigned)(nv * bpv)), dim3(256), 0, s, X, n, bpv, part);
  std::vector<double> ph((size_t)nv * bpv), out(nv, 0.0);
  BW_HIP(hipMemcpyAsync(ph.data(), part, ph.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  for (int v = 0; v < nv; ++v)
    for (int b = 0; b < bpv; ++b) out[v] += ph[(size_t)v * bpv + b];
  return out;
}

template <typename T>
int effective_stiffness(bw_rve* r, double rtol, int maxit, double* Ceff, int32_t* iters, hipStream_t s) {
  const Geom& g = r->g;
  const long N = g.nvox;
  const int bpv = 64;
  char* base = (char*)r->ws_misc.get((size_t)72 * N * sizeof(cplx<T>) + (size_t)6 * bpv * 6 * sizeof(double));
  cplx<T>* S = (cplx<T>*)base;   // 6 x 6 fields: unit stresses, then strains
  cplx<T>* B = S + 36 * N;       // 6 x 3 right-hand sides
  cplx<T>* X = B + 18 * N;       // 6 x 3 fluctuations
  double* part = (double*)(X + 18 * N);
  hipLaunchKernelGGL((k_unit_stress<T>), dim3(grid_of(N)), dim3(256), 0, s, (const uint16_t*)r->d_gmap, ctab<T>(r), S,
                     N);
  fft3_nc<T, false>(r, S, 6, 6, s);
  const double k0[18] = {0};
  QTable qt = make_qtable(r, k0, 1);
  const double* dq = upload_qtable(r, qt, r->ws_q3, s);
  hipLaunchKernelGGL((k_div_hat<T>), dim3(grid_of(6 * N)), dim3(256), 0, s, (const cplx<T>*)S, dq, B, g.n0, g.n1, g.n2,
                     N, 6, 1.0);
  // A right-hand side at the rounding level of its stress (a homogeneous cell: the
  // transform of a uniform stress vanishes off xi = 0 up to rounding) is zero: its
  // fluctuation is 0, which a tolerance relative to the noise itself cannot reach.
  {
    double qm2 = 0;
    const int nax[3] = {g.n0, g.n1, g.n2};
    for (int a = 0, o = 0; a < 3; o += nax[a], ++a) {
      double m = 0;
      for (int i = 0; i < nax[a]; ++i) m = std::max(m, qt.host[o + i] * qt.host[o + i]);
      qm2 += m;
    }
    const double eps = 1e3 * std::numeric_limits<T>::epsilon();
    const std::vector<double> ns = field_norms2<T>(S, 6, 6 * N, part, bpv, s);
    const std::vector<double> nb = field_norms2<T>(B, 6, 3 * N, part, bpv, s);
    for (int j = 0; j < 6; ++j)
      if (nb[j] <= eps * eps * qm2 * ns[j])
        BW_HIP(hipMemsetAsync(B + (size_t)j * 3 * N, 0, (size_t)3 * N * sizeof(cplx<T>), s));
  }
  const double* q6 = upload_qtable(r, make_qtable(r, k0, 6), r->ws_q2, s);
  PcgResult res = pcg_run<T>(r, q6, qt, B, X, 6, rtol, maxit, true, s);
  if (qt.null_index[0] >= 0) zero_voxel<T>(X, 6, N, qt.null_index[0], s);
  hipLaunchKernelGGL((k_strain_hat<T>), dim3(grid_of(6 * N)), dim3(256), 0, s, (const cplx<T>*)X, dq, S, g.n0, g.n1,
                     g.n2, N, 6, 1.0);
  fft3_nc<T, true>(r, S, 6, 6, s);
  hipLaunchKernelGGL((k_mean_stress<T>), dim3(6 * bpv), dim3(256), 0, s, (const uint16_t*)r->d_gmap, ctab<T>(r),
                     (const cplx<T>*)S, N, 1.0 / (double)N, bpv, part);
  std::vector<double> ph((size_t)6 * bpv * 6);
  BW_HIP(hipMemcpyAsync(ph.data(), part, ph.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  BW_HIP(hipStreamSynchronize(s));
  double Cs[6][6];
  for (int j = 0; j < 6; ++j)
    for (int a = 0; a < 6; ++a) {
      double t = 0;
      for (int b = 0; b < bpv; ++b) t += ph[((size_t)j * bpv + b) * 6 + a];
      Cs[a][j] = t / (double)N;
    }
  for (int a = 0; a < 6; ++a)
    for (int j = 0; j < 6; ++j) Ceff[a * 6 + j] = 0.5 * (Cs[a][j] + Cs[j][a]) * r->Cref;
  for (int v = 0; v < 6; ++v)
    if (iters) iters[v] = res.iters[v];
  if (!res.converged) {
    set_error("homogenization: some cell problem did not reach the tolerance within maxit");
    return BW_ENOTCONV;
  }
  return BW_OK;
}

}  // namespace

extern "C" int bw_mode_fields(bw_rve* r, const double k[3], int32_t nmodes, const void* modes, void* u_out,
                              void* eps_out, double* phase_host, void* stream) {
  try {
    BW_REQUIRE(r && k, BW_EINVAL, "null argument");
    BW_REQUIRE(nmodes >= 0, BW_EINVAL, "nmodes < 0");
    for (int a = 0; a < 3; ++a) BW_REQUIRE(std::isfinite(k[a]), BW_EINVAL, "non-finite wave vector");
    if (nmodes == 0) return BW_OK;
    BW_REQUIRE(modes && u_out, BW_EINVAL, "null argument");
    BW_REQUIRE(modes != u_out && (!eps_out || (eps_out != modes && eps_out != u_out)), BW_EINVAL,
               "modes, u_out and eps_out must not alias");
    hipStream_t s = (hipStream_t)stream;
    if (r->precision == BW_FP64)
      mode_fields<double>(r, k, nmodes, (const cplx<double>*)modes, (cplx<double>*)u_out, (cplx<double>*)eps_out,
                          phase_host, s);
    else
      mode_fields<float>(r, k, nmodes, (const cplx<float>*)modes, (cplx<float>*)u_out, (cplx<float>*)eps_out,
                         phase_host, s);
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

extern "C" int bw_effective_stiffness(bw_rve* r, double rtol, int32_t maxit, double* C66_host, int32_t* iters_host,
                                      void* stream) {
  try {
    BW_REQUIRE(r && C66_host, BW_EINVAL, "null argument");
    BW_REQUIRE(rtol >= 0 && rtol < 1, BW_EINVAL, "rtol must be in [0, 1)");
    if (rtol == 0) rtol = r->precision == BW_FP64 ? 1e-12 : 1e-6;
    if (maxit <= 0) maxit = 20000;
    hipStream_t s = (hipStream_t)stream;
    const int code = r->precision == BW_FP64 ? effective_stiffness<double>(r, rtol, maxit, C66_host, iters_host, s)
                                             : effective_stiffness<float>(r, rtol, maxit, C66_host, iters_host, s);
    BW_HIP(hipGetLastError());
    return code;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal: ") + e.what());
    return BW_EINVAL;
  }
}
