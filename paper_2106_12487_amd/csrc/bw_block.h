// Block kernels of the eigen-solvers: Gram products on FP64 MFMA, Ritz
// updates, batched inner products, the small generalized Hermitian
// eigenproblem (single workgroup, FP64), Gamma-point deflation and vector
// utilities.  Blocks of vectors are stored vector-major: vector p starts at
// X + p * vstride (complex elements), each of length n.
#pragma once
#include "bw_internal.h"

namespace bw {

constexpr int GRAM_QMAX = 32;  // Gram / Ritz block limit
constexpr int GEIG_QMAX = 48;  // small eigenproblem limit

// G[i][j] = sum_e conj(X_i[e]) Y_j[e], i < qx, j < qy  (FP64, deterministic)
template <typename T>
void launch_gram(const cplx<T>* X, int qx, const cplx<T>* Y, int qy, long n, long vstride, double2* G,
                 DevBuf& scratch, unsigned* counter, hipStream_t s);
// Y_j = sum_p X_p Q[p][j], j < qout (Q is q x q row-major, FP64).  real_q: Q
// is real (its imaginary parts are ignored), half the multiply-adds.
template <typename T>
void launch_ritz(const cplx<T>* X, int q, const double2* Q, int ldq, cplx<T>* Y, int qout, long n, long vstride,
                 hipStream_t s, bool real_q = false);
// out[p] = <X_p, Y_p> (complex, FP64) for p < nv
template <typename T>
void launch_dots(const cplx<T>* X, const cplx<T>* Y, int nv, long n, long vstride, double2* out, DevBuf& scratch,
                 unsigned* counters, hipStream_t s);
// R_p = A_p - lam_p B_p (lam device, FP64)
template <typename T>
void launch_lincomb(const cplx<T>* A, const cplx<T>* B, const double* lam, cplx<T>* R, int nv, long n, long vstride,
                    hipStream_t s);
// Y_p = s_p X_p (s device)
template <typename T>
void launch_scale_cols(const cplx<T>* X, const double* sc, cplx<T>* Y, int nv, long n, long vstride, hipStream_t s);
// dst (TD) = src (TS)
template <typename TS, typename TD>
void launch_convert(const cplx<TS>* src, cplx<TD>* dst, size_t n, hipStream_t s);
// M-orthogonal projection off the rigid translations for (X, MX) pairs; MN are
// the three vectors M e_{j*,c}; coefficients a_c = MX_p(c, j*) (M n_c is 1 at j*).
template <typename T>
void launch_deflate(cplx<T>* X, cplx<T>* MX, const cplx<T>* MN, int nv, long nvox, long jstar, double2* coef,
                    hipStream_t s);
// plane-wave start vectors: vector p = pol[p] at voxel vox[p] (others zero)
template <typename T>
void launch_planewaves(cplx<T>* U, int nv, long nvox, const long* vox, const double* pol, hipStream_t s);
// Per-k bases (batched Lanczos): basis vector i of wave vector k sits at
// X + k * xk + i * xi; the batch vector of k at Y + k * yk.
// out0[k * ldo + i] = <X_k[i], Y0_k>, out1[k * ldo + i] = <X_k[i], Y1_k> for i < J,
// each basis vector read once
template <typename T>
void launch_mdot2(const cplx<T>* X, long xk, long xi, int J, const cplx<T>* Y0, long yk0, const cplx<T>* Y1, long yk1,
                  int nk, long n, const int* act, double2* out0, double2* out1, int ldo, DevBuf& scratch,
                  hipStream_t s);
// Y0_k <- f0 Y0_k - sum_i X_k[i] a_i;  Y1_k <- f1 Y1_k - sum_i X_k[i] b_i - g Y0_k(new)
// (coefficients at c + k * ldc: a[0..J-1], b[0..J-1], (f0, 0), (f1, 0), g; Y1 may be null)
template <typename T>
void launch_mlincomb2(cplx<T>* Y0, long yk0, cplx<T>* Y1, long yk1, const cplx<T>* X, long xk, long xi, int J,
                      const double2* c, int ldc, int nk, long n, const int* act, hipStream_t s);
// Y_k = sc[k] * X_k with independent strides
template <typename T>
void launch_scale_copy(const cplx<T>* X, long xk, cplx<T>* Y, long yk, const double* sc, int nk, long n,
                       const int* act, hipStream_t s);

// U[vec[e] * vstride + c * nvox + vox[e]] = val[3 e + c] (real) for e < nent
// (added to the entry when `add`); the (vec, vox) pairs must be distinct
template <typename T>
void launch_set_entries(cplx<T>* U, long vstride, long nvox, int nent, const long* vec, const long* vox,
                        const double* val, hipStream_t s, bool add = false);

// X_p += amp * (u1 + i u2), u uniform in [-1, 1) from a counter hash of (seed, p, e)
template <typename T>
void launch_add_hash(cplx<T>* X, long n, long vstride, int nv, unsigned long long seed, double amp, hipStream_t s);

// small generalized Hermitian eigenproblem Kq z = lam Mq z (q <= GEIG_QMAX):
// lam ascending, Q with Q^H Mq Q = I.  info[0] != 0 if Mq is not positive definite.
void launch_small_geig(const double2* Kq, const double2* Mq, int q, double* lam, double2* Q, int* info,
                       hipStream_t s);
// nb independent Hermitian eigenproblems H_b z = lam z (q x q each, stored one
// after the other), one workgroup each: lam[b*q..], Q[b*q*q..], info[b]
void launch_small_eig_batched(const double2* H, int q, int nb, double* lam, double2* Q, int* info, hipStream_t s);

}  // namespace bw
