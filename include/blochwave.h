/*
 * blochwave.h -- C ABI of the MI355X (gfx950) implementation of the FFT-based
 * Bloch-wave method of Segurado & Lebensohn ("An FFT-based approach for Bloch
 * wave analysis: application to polycrystals").
 *
 * Problem (Sec. 3.2, eqs. hatA, hatM, eigen_fourier_3D): for a voxelized
 * periodic cell with stiffness C(x) and density rho(x), find the lowest
 * eigenpairs of  K(k) U^ = omega^2 M U^  at each Bloch wave vector k, with
 *   K(k) U^ = (xi_j + k_j) F{ C_ijkl(x) F^-1[(xi_l + k_l) U^_k] },
 *   M U^    = F{ rho(x) F^-1[U^] }.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units      SI throughout (Pa, kg/m^3, m, rad/m, rad/s).
 * Grid       n[0] x n[1] x n[2] voxels, C order (n[2] fastest), cell edges L[3].
 * Vectors    Fourier coefficients of the periodic displacement, layout
 *            [nvec][3][n0][n1][n2] of interleaved complex numbers: double2 when
 *            the cell was created with BW_FP64, float2 with BW_MIXED.  The
 *            forward DFT is unnormalized, U^(m) = sum_x U(x) exp(-2 pi i j.m/n);
 *            storage index j holds the frequency label m = j (mod n) taken from
 *            the window of Sec. 3.1 eq. "frequencies" (Nyquist label -n/2),
 *            shifted by whole reciprocal vectors so that the reduced wave number
 *            k_a L_a / 2 pi - shift lies in (-1/2, 1/2].  For k in the first
 *            Brillouin zone this is exactly the paper's window.
 * Stiffness  per grain, 21 entries of the 6x6 Voigt matrix (engineering shear
 *            strain [e11, e22, e33, 2e23, 2e13, 2e12]), upper triangle,
 *            row-major, in the sample frame.
 * Counts     a zero count (nvec, nrhs, nk, nmodes where the call allows 0) is a
 *            no-op that returns 0; the buffers it would address may then be
 *            NULL.
 * Memory     pointers named *_host are host memory; all vector arguments are
 *            device memory owned by the caller.  The library owns only what
 *            bw_create_rve allocates (freed by bw_destroy_rve) plus cached
 *            workspaces attached to the cell.  It never frees caller memory.
 * Streams    `stream` is a hipStream_t (NULL = the default stream).  Operator
 *            calls are asynchronous on it; calls returning host results
 *            synchronize it before returning.
 * Errors     0 = success; < 0 = error, outputs undefined (BW_EINVAL bad
 *            argument, BW_ENOMEM allocation failed, BW_EHIP a HIP runtime
 *            error, BW_EUNSUPPORTED grid size without a compiled FFT);
 *            > 0 = warning with valid outputs (BW_ENOTCONV an iteration hit its
 *            limit, results carry their error bounds; BW_ESTALL the learned
 *            preconditioner stalled and the solve finished with the plain one).
 *            bw_last_error() returns a thread-local message for the last non-zero
 *            status.
 * Threads    a cell handle is not thread-safe; different handles may be used
 *            concurrently on different streams.
 */
#ifndef BLOCHWAVE_H
#define BLOCHWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BW_OK 0
#define BW_ENOTCONV 1
#define BW_ESTALL 2
#define BW_EINVAL (-1)
#define BW_ENOMEM (-2)
#define BW_EHIP (-3)
#define BW_EUNSUPPORTED (-4)

/* working precision of a cell */
#define BW_FP64 0   /* FFTs, contraction and vectors in double              */
#define BW_MIXED 1  /* FFTs, contraction and PCG vectors in float; FP64
                       reductions, Rayleigh-Ritz and eigen-residuals        */

/* eigen-solver */
#define BW_SUBSPACE 0 /* Sec. 3.3, Algorithm "subspace" (Bathe), block PCG   */
#define BW_LANCZOS 1  /* Sec. 3.3, shift-invert restarted Lanczos           */

typedef struct bw_rve bw_rve;
typedef struct bw_unet bw_unet;   /* the learned preconditioner (below) */

/* preconditioner of the inner solves */
#define BW_PLAIN 0    /* P(C0, xi + k)^-1 of the homogeneous reference medium (Sec. 3.3) */
#define BW_LEARNED 1  /* plus the network correction, in flexible PCG (bw_pcg_solve_learned) */

/* Options of bw_lowest_modes.  Zero-initialized fields take the defaults shown. */
typedef struct bw_eig_opts {
  int32_t method;      /* BW_SUBSPACE (default) or BW_LANCZOS                    */
  int32_t block;       /* subspace block q; 0 -> min(2 nmodes, nmodes + 8)       */
  int32_t ncv;         /* Lanczos basis size; 0 -> max(2 nw + 1, 20), nw = nmodes,
                          or nmodes - 3 (the rigid translations are not sought)
                          when every wave vector of the batch is Gamma-like      */
  int32_t maxit_outer; /* outer iterations / restarts per k; 0 -> 200            */
  int32_t maxit_lin;   /* PCG iterations per solve; 0 -> 20000                   */
  int32_t warm_start;  /* subspace: start k from the previous k's Ritz block     */
  double tol_eig;      /* eigen tolerance TOL_eig; 0 -> 1e-10                    */
  double tol_lin;      /* PCG relative tolerance TOL_lin; 0 -> 1e-10 (FP64),
                          1e-6 (MIXED inner solves)                              */
  double tol_omega;    /* > 0: stop a wave vector as soon as every wanted mode
                          carries an a-posteriori bound on its relative omega
                          error <= tol_omega (with the subspace method the inner
                          PCG tolerance then adapts to the outer residual, never
                          looser than 1e-2 nor tighter than tol_lin; Lanczos
                          keeps tol_lin); 0: the err1 / err2 rule of the
                          subspace algorithm with TOL_eig                        */
  int32_t kbatch;      /* Lanczos: wave vectors advanced together (one PCG right-
                          hand side each per Lanczos step); 0 -> as many as fit
                          in about 48 GB, at most 64; 1 -> one k at a time.
                          Every step is per wave vector (the start vector's
                          pseudo-random part is seeded by k itself), so a wave
                          vector's results do not depend on kbatch or on the
                          other wave vectors of the call, except that with
                          ncv = 0 a batch of Gamma-like wave vectors only gets
                          the shorter default basis of nmodes - 3 wanted modes */
  int32_t precond;     /* BW_PLAIN (default) or BW_LEARNED: the Lanczos inner
                          solves of a BW_MIXED cell by flexible PCG with `net`
                          (grids multiple of 4; the FP64 refinement keeps P^).
                          A right-hand side whose learned steps stall finishes
                          with P^ and the call returns BW_ESTALL (valid results) */
  const bw_unet* net;  /* the network for BW_LEARNED                              */
  int32_t group_cells; /* bw_lowest_modes_batched with BW_LANCZOS: 0 (default) ->
                          every cell runs on a stream of its own; 1 -> cells of
                          one grid, cell edge and precision form a group whose
                          wave vectors share every batched launch (each vector
                          with its own cell's grain map and reference stiffness;
                          at most 8 cells per group; not when modes are
                          requested or with BW_LEARNED)                        */
  int32_t kgroups;     /* BW_LANCZOS with BW_PLAIN on a single cell: the wave
                          vectors are split into this many groups (at most 8;
                          wave vector i in group i mod kgroups) solved
                          concurrently, each on a stream and
                          host thread of its own with workspaces of its own (the
                          cell's tables are shared), so that one group's
                          latency-bound transforms overlap another's memory-
                          bound steps; a wave vector's results are those of one
                          batch bit for bit.  0 or 1 -> one group            */
} bw_eig_opts;

/* Statistics of the last solver call (all optional outputs). */
typedef struct bw_stats {
  int64_t pcg_iterations;   /* sum over right-hand sides of PCG iterations      */
  int64_t block_iterations; /* batched PCG sweeps (each sweep = one K apply of
                               the whole block)                                 */
  int64_t outer_iterations; /* subspace iterations / Lanczos restarts            */
  int64_t k_applies;        /* single-vector K applies, all precisions          */
  int64_t m_applies;        /* single-vector M applies                          */
  double seconds;           /* wall time of the call                            */
} bw_stats;

/* Create a cell (Sec. 3.2; Algorithm "Full algorithm" step (a)).
 *   out            receives the handle
 *   n[3], L[3]     grid and cell edges (n[i] >= 1, L[i] > 0)
 *   grain_map_host n0*n1*n2 uint16 grain index per voxel (C order)
 *   n_grains       number of grains G (1 .. 65535)
 *   C21_host       G x 21 Voigt stiffness per grain (see Conventions); each
 *                  6x6 matrix must be symmetric positive definite
 *   rho_host       G densities (> 0)
 *   precision      BW_FP64 or BW_MIXED
 * The volume-averaged stiffness C0 used by the preconditioner (Sec. 3.3 eq.
 * precond) and the mean density are computed here.  Returns BW_EINVAL on bad
 * input, BW_EUNSUPPORTED if a grid size has no compiled FFT length. */
int bw_create_rve(bw_rve** out, const int32_t n[3], const double L[3],
                  const uint16_t* grain_map_host, int32_t n_grains,
                  const double* C21_host, const double* rho_host, int32_t precision,
                  void* stream);

/* Release the cell and every workspace the library allocated for it. */
void bw_destroy_rve(bw_rve* rve);

/* FFT schedule autotuner: for each axis, times bw_apply_K on nvec vectors
 * (1 .. 256) with the register-resident kernels (power-of-two lengths 16 ..
 * 256) and with the generic LDS kernels at the widest tile and at 1/2 and 1/4
 * of it, and keeps the fastest for this cell (used by every later operator
 * apply and PCG; results agree to rounding whatever the schedule).
 * speedup_host (optional) receives time(default schedule) / time(chosen).
 * A BW_MIXED cell also gets a schedule of its own for its FP64 applies (the
 * Rayleigh-Ritz refinement), timed on min(nvec, 16) FP64 vectors.
 * Allocates and frees two scratch blocks of nvec vectors.  Synchronizes `stream`. */
int bw_autotune(bw_rve* rve, int32_t nvec, double* speedup_host, void* stream);

/* Get (set = 0) or set (set != 0) the FFT schedule of a cell per axis 0..2:
 * reg[a] != 0 uses the register kernels where the length allows, cap[a] > 0
 * limits the lines per tile of the generic kernels (0 = as many as fit).  Set
 * applies to the FP32 and FP64 kernels alike; get returns the schedule of the
 * cell's main precision (FP32 for BW_MIXED). */
int bw_fft_schedule(bw_rve* rve, int32_t reg[3], int32_t cap[3], int32_t set);

/* Query grid / precision / volume averages of a cell.  Any output may be NULL. */
int bw_rve_info(const bw_rve* rve, int32_t n[3], int32_t* precision, double C0_21[21],
                double* rho_bar);

/* y = K(k) u for nvec vectors (Sec. 3.2 eq. hatA).  k_host: 3 doubles (rad/m).
 * u and y: device [nvec][3][n0][n1][n2] complex in the cell's precision; they
 * must not alias. */
int bw_apply_K(bw_rve* rve, const double k_host[3], const void* u, void* y, int32_t nvec,
               void* stream);

/* y = K(k) u exactly as bw_apply_K (same kernels, same results), for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops): the call allocates nothing.  Its work array (6 nvec n0 n1 n2 complex
 * numbers in the cell's precision, rounded up to 256 bytes) and its table of
 * shifted wave numbers (nvec (n0 + n1 + n2) doubles) live in a scratch area of
 * the library of BW_NOALLOC_SCRATCH_BYTES (64 MiB) in each device's memory,
 * held until the process ends; larger requests return BW_EINVAL (e.g. FP32 at
 * 64^3: up to 5 vectors; at 128^3 none).  Every call on a device uses that
 * device's one area: calls that overlap on one device (concurrent streams or
 * threads) race and give wrong results.  The cell must already exist (its
 * tables are allocated by bw_create_rve), and kernel timing must be off (it
 * creates events). */
#define BW_NOALLOC_SCRATCH_BYTES (64u << 20)
int bw_apply_K_noalloc(bw_rve* rve, const double k_host[3], const void* u, void* y, int32_t nvec,
                       void* stream);

/* y = M u (Sec. 3.2 eq. hatM).  Same layout rules as bw_apply_K. */
int bw_apply_M(bw_rve* rve, const void* u, void* y, int32_t nvec, void* stream);

/* y = P^ u, the homogeneous-reference preconditioner P(C0, xi + k)^-1 applied
 * per Fourier voxel (Sec. 3.3 eqs. matrixP, precond); zero where xi + k = 0. */
int bw_apply_P(bw_rve* rve, const double k_host[3], const void* u, void* y, int32_t nvec,
               void* stream);

/* Solve K(k) x = b for nrhs right-hand sides by preconditioned CG
 * (Sec. 3.3, Algorithm "InvA"), stopping when the true residual satisfies
 * ||K x - b|| <= rtol ||b|| (Euclidean norm of the DFT coefficients).
 *   b, x       device [nrhs][3][n0][n1][n2]; x holds the initial guess on entry
 *              and the solution on exit; b is not modified
 *   maxit      iteration limit per right-hand side (<= 0: 20000)
 *   iters_host optional int32[nrhs]: iterations used
 *   relres_host optional double[nrhs]: final true relative residual, computed
 *              in the working precision with FP64 accumulation
 * When xi + k = 0 for some voxel (k a reciprocal lattice vector) K is singular;
 * the component of b on that voxel must be zero (BW_EINVAL otherwise) and the
 * solution is returned with that component zero.  Returns BW_ENOTCONV if some
 * right-hand side hit maxit.  Synchronizes `stream`. */
int bw_pcg_solve(bw_rve* rve, const double k_host[3], const void* b, void* x, int32_t nrhs,
                 double rtol, int32_t maxit, int32_t* iters_host, double* relres_host,
                 void* stream);

/* Lowest nmodes eigenpairs of K(k) U = omega^2 M U at nk wave vectors
 * (Algorithm "Full algorithm"; eigen-solver per opts->method).
 *   k_list_host  nk x 3 doubles (rad/m), processed in order (warm starts follow it)
 *   omega_host   nk x nmodes doubles, ascending per k (rad/s)
 *   err_host     optional nk x nmodes: a-posteriori bound on |omega - omega*| /
 *                omega* from the FP64 eigen-residual (Kato-Temple when the gap
 *                to the next Ritz value allows it, else the residual bound)
 *   modes        optional device nk x nmodes x [3][n0][n1][n2] complex in the
 *                cell's precision, M-normalized (U^H M U = 1)
 *   stats_host   optional solver statistics
 * At k = 0 (mod reciprocal lattice) the three rigid translations are returned
 * as omega = 0 with constant M-normalized modes and the rest is solved on their
 * M-orthogonal complement.  BW_LANCZOS advances one Krylov vector per wave
 * vector, so an exactly degenerate eigenvalue (homogeneous cells, symmetric
 * cells at symmetric k) is found once; BW_SUBSPACE (a block method) resolves
 * such multiplicities.  BW_LANCZOS needs ncv <= 3 n0 n1 n2 - 3 (the dimension
 * of the Krylov space without the rigid translations) and returns BW_EINVAL on
 * smaller cells.  Synchronizes `stream`. */
int bw_lowest_modes(bw_rve* rve, const double* k_list_host, int32_t nk, int32_t nmodes,
                    const bw_eig_opts* opts, double* omega_host, double* err_host,
                    void* modes, bw_stats* stats_host, void* stream);

/* Lowest modes of several cells at once (uneven grids allowed; Algorithm
 * "Full algorithm" per cell): cell i gets nks[i] wave vectors k_lists[i]
 * (host, nks[i] x 3) and writes omegas[i] / errs[i] (host, nks[i] x nmodes;
 * errs and modes may be NULL, as may any errs[i] / modes[i]) exactly as a
 * separate bw_lowest_modes call would.  The cells advance concurrently, each
 * on a stream of its own created by the library, from host threads of the
 * library, so the kernels of small cells overlap on the GPU; every cell's
 * results equal those of its own call (same kernels, deterministic
 * reductions).  The call first waits for `stream` and returns when all cells
 * are done.  stats (optional) sums the counters over the cells; its
 * `seconds` is the wall time of the whole call.  Returns the most severe
 * status of the cells (an error before BW_ENOTCONV); bw_last_error names the
 * first failing cell.  Different cells must be different handles; nrve <= 256. */
int bw_lowest_modes_batched(bw_rve* const* rves, int32_t nrve, const double* const* k_lists, const int32_t* nks,
                            int32_t nmodes, const bw_eig_opts* opts, double* const* omegas, double* const* errs,
                            void* const* modes, bw_stats* stats, void* stream);

/* Diagnostics: opt-in kernel timing.  bw_timing_enable(1) clears the totals
 * and brackets every subsequent kernel launch of the library with HIP events
 * on the launch stream; bw_timing_enable(0) stops recording.  Adds a few
 * microseconds of event overhead per launch. */
int bw_timing_enable(int32_t enable);

/* PCG iterations run as captured HIP graphs (one graph per chunk of iterations
 * between host convergence checks, captured once per cell and buffer set and
 * replayed) unless disabled here or while kernel timing is enabled.  Default:
 * enabled.  Results are identical either way (same kernels, same order). */
int bw_graphs_enable(int32_t enable);

/* Restricts the timing to the kernel of that name (NULL or "" = all kernels). */
int bw_timing_filter(const char* kernel_name);

/* Writes a JSON object {"kernel": {"launches": n, "ms": total, "units": u,
 * "union_ms": w}} into buf (len bytes, NUL-terminated, truncated if needed)
 * after waiting for the recorded events; `units` counts the vectors each kernel
 * processed, `ms` sums the launch durations and `union_ms` is the time during
 * which at least one launch of the kernel ran (less than `ms` when launches on
 * concurrent streams overlap).  Returns the length the full report needs
 * (including the NUL). */
int64_t bw_timing_report(char* buf, int64_t len);

/* ------------------------------------------------------------------------
 * Learned preconditioner (an extension of the homogeneous-reference
 * preconditioner of Sec. 3.3 eqs. matrixP, precond; not part of the paper).
 *
 *   z = P^ r + F[ s e^{i phi} N_theta(x) ],
 *   x = [ e^{-i phi} F^-1(P^ r) / s  (real and imaginary parts of the three
 *         components: 6 channels),  the 21 scaled Voigt stiffness entries and
 *         the scaled density of the voxel's grain (22 channels) ]
 * in real space, with s the RMS of F^-1(P^ r) over voxels and components and
 * phi = arg(sum of (F^-1 P^ r)^2) / 2.  N_theta is a 3-level 3D U-Net
 * (16 / 32 / 64 channels, 3x3x3 periodic convolutions, ReLU, 2x2x2 average
 * pooling, nearest upsampling with skip concatenation, 1x1x1 head), evaluated
 * with BF16 matrix-core products and FP32 accumulation.  Every grid size must
 * be a multiple of 4 (BW_EUNSUPPORTED otherwise) and the cell BW_MIXED.
 *
 * Parameters: one flat FP32 vector, per layer l = 0..8 the weights
 * W_l[tap][c_out][c_in] followed by the bias b_l[c_out]; layers
 * (c_in -> c_out, taps): 32->16 (27), 16->16 (27), 16->32 (27), 32->32 (27),
 * 32->64 (27), 64->64 (27), 96->32 (27), 48->16 (27), 16->16 (1).  Tap
 * t = 9 (d0 + 1) + 3 (d1 + 1) + (d2 + 1) reads the periodic neighbour at grid
 * offset (d0, d1, d2), d in {-1, 0, 1}.  Input channels 28..31 of layer 0 and
 * output channels 6..15 of layer 8 are padding: their weights are held at 0.
 * Concatenations put the upsampled coarse channels first, then the skip.
 * ------------------------------------------------------------------------ */
/* Number of FP32 parameters of the network. */
int64_t bw_unet_param_count(void);

/* Create a network on the current device: He-normal weights from `seed`, zero
 * biases and a zero head (the untrained network adds nothing to P^ r). */
int bw_unet_create(bw_unet** out, uint64_t seed);

/* Release the network and its workspaces. */
void bw_unet_destroy(bw_unet* net);

/* Copy the FP32 parameters to / from host memory (n = bw_unet_param_count()).
 * Setting weights zeroes the padding entries, checks that every value is
 * finite (BW_EINVAL otherwise) and resets the optimizer state. */
int bw_unet_get_weights(const bw_unet* net, float* w_host, int64_t n);
int bw_unet_set_weights(bw_unet* net, const float* w_host, int64_t n);

/* The bare network on nb samples of an n[0] x n[1] x n[2] grid:
 *   x  device float [nb][n0*n1*n2][32] (channels last), y device float
 *      [nb][n0*n1*n2][16].  Asynchronous on `stream`. */
int bw_unet_net_forward(bw_unet* net, const int32_t n[3], const float* x, float* y, int32_t nb, void* stream);

/* Gradient of sum(dy . y(x)) with respect to the parameters, written to
 * grad_host (bw_unet_param_count() floats; padding entries 0).  x and dy are
 * device buffers laid out as in bw_unet_net_forward.  Synchronizes `stream`. */
int bw_unet_net_backward(bw_unet* net, const int32_t n[3], const float* x, const float* dy, float* grad_host,
                         int32_t nb, void* stream);

/* z = learned preconditioner applied to nrhs residuals r of the physical
 * system K(k) x = r (k_host: nrhs x 3, one wave vector per right-hand side);
 * r, z device [nrhs][3][n0][n1][n2] float2, not aliased.  The component on
 * the xi + k = 0 voxel (if any) is zero.  Synchronizes `stream`. */
int bw_unet_apply(bw_unet* net, bw_rve* rve, const double* k_host, const void* r, void* z, int32_t nrhs,
                  void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * mean squared error between N_theta(x) and the normalized real-space target
 * e^{-i phi} F^-1(x* - P^ r) / s, over nrhs pairs (r, x* = K(k)^-1 r) of
 * device vectors laid out as in bw_unet_apply.  loss_host (optional) receives
 * the loss before the step.  Synchronizes `stream`. */
int bw_unet_train_step(bw_unet* net, bw_rve* rve, const double* k_host, const void* r, const void* x_star,
                       int32_t nrhs, double lr, double* loss_host, void* stream);

/* One Adam step (as bw_unet_train_step) on the residual loss
 *   mean over the nrhs residuals of ||K(k) z - r||^2 / ||r||^2,
 * z the learned preconditioner applied to r (Euclidean norms of the Fourier
 * coefficients; the gradient through K is one more K apply, K being Hermitian).
 * Needs no solutions: the pairs are residuals alone, e.g. those of plain PCG
 * iterates.  loss_host (optional) receives the loss before the step.
 * Synchronizes `stream`. */
int bw_unet_train_step_residual(bw_unet* net, bw_rve* rve, const double* k_host, const void* r, int32_t nrhs,
                                double lr, double* loss_host, void* stream);

/* Solve K(k) x = b by flexible preconditioned CG with the learned
 * preconditioner (net may be NULL: the plain P^, which reproduces
 * bw_pcg_solve's iterates up to rounding).  Directions are made K-orthogonal
 * to the previous one (Polak-Ribiere form, needed for a nonlinear
 * preconditioner).  Per right-hand side, a learned z with Re <r, z> <= 0 or a
 * non-finite value is replaced by P^ r and the direction restarted; after
 * three such events, or when the residual has not dropped by 10% over 10
 * iterations, the right-hand side continues with P^ only.  Arguments as in
 * bw_pcg_solve (BW_MIXED cells, float2 vectors); fallbacks_host (optional,
 * int32[nrhs]) receives the number of fallback events.  Synchronizes `stream`. */
int bw_pcg_solve_learned(bw_rve* rve, bw_unet* net, const double k_host[3], const void* b, void* x, int32_t nrhs,
                         double rtol, int32_t maxit, int32_t* iters_host, double* relres_host,
                         int32_t* fallbacks_host, void* stream);

/* ---------------------------------------------------------------------------
 * Dispersion post-processing (Sec. 5.1)
 * --------------------------------------------------------------------------- */

/* Slopes d omega / ds of the branches along the direction dir (any nonzero
 * vector; normalized here) at the wave vector k_host (rad/m): the group
 * velocity of Sec. 5.1 eq. c_group projected on dir.  modes: device, the
 * nmodes (1 .. 32) eigenvectors at k_host as written by bw_lowest_modes for this
 * cell (complex128 for BW_FP64 cells, complex64 for BW_MIXED ones), omega_host
 * their frequencies (rad/s, ascending, >= 0).  Computed in FP64 from
 * D = U^H dK/ds U (exact from two K applies, since K is quadratic in k) and
 * U^H M U: a mode whose omega is separated from its neighbours by more than
 * cluster_tol (relative) gets D_pp / (2 omega U_p^H M U_p); within a cluster of
 * equal omega the slopes are the eigenvalues of (D, U^H M U) on the cluster over
 * 2 omega, ascending (they do not depend on the basis the modes came in).
 * Modes with omega = 0 (rigid translations at Gamma) get 0.  slopes_host:
 * float64[nmodes] (m/s).  Synchronizes `stream`.  BW_EINVAL on bad arguments. */
int bw_group_velocity(bw_rve* rve, const double k_host[3], const double dir[3], int32_t nmodes,
                      const void* modes, const double* omega_host, double cluster_tol,
                      double* slopes_host, void* stream);

/* Long-wave speeds of the three acoustic branches along dir (m/s, ascending):
 * omega / |k| from bw_lowest_modes (subspace iteration, bound-based stopping at
 * tol_omega; 0 -> 1e-10 for BW_FP64, 1e-8 for BW_MIXED) at k = +-h dir and
 * +-2h dir with h = h_frac pi / max(L) (h_frac in (0, 0.25]), c(h) the mean
 * of omega / |k| over +-k (even in k also on even grids, whose frequency set
 * is not symmetric), extrapolated to k -> 0 as (4 c(h) - c(2h)) / 3.  The
 * limit is the speed of the equivalent homogeneous medium (Sec. 5.1).  Returns
 * the status of the eigen-solve (BW_ENOTCONV with c_host filled when a bound
 * missed tol_omega).  Synchronizes `stream`. */
int bw_long_wave_speeds(bw_rve* rve, const double dir[3], double h_frac, double tol_omega, double* c_host,
                        void* stream);

/* Real-space fields of modes at k (Sec. 5.2, eigenvectors, eq. rotate_eigenvector):
 * u = e^{-i phi} F^-1(U^) with the inverse DFT normalized by 1/N and
 * phi = arg(sum_x u . u) / 2 (the phase that brings the field closest to real;
 * for a field of common phase it is that phase, up to pi; 0 when the sum
 * vanishes), and the strain eps = e^{-i phi} F^-1[i B(xi + k) U^] (Voigt order
 * 11, 22, 33, 23, 13, 12, engineering shear; the strain of the Bloch wave
 * u(x) e^{i k.x} divided by e^{i k.x}).  Grid point i sits at x = i L / n.
 * modes: device [nmodes][3][n0][n1][n2] complex in the cell's precision (as
 * bw_lowest_modes writes them); u_out: device, same shape; eps_out: optional
 * device [nmodes][6][n0][n1][n2]; phase_host: optional float64[nmodes].  No
 * argument may alias another.  Synchronizes `stream`. */
int bw_mode_fields(bw_rve* rve, const double k_host[3], int32_t nmodes, const void* modes, void* u_out,
                   void* eps_out, double* phase_host, void* stream);

/* Effective stiffness of the cell by static homogenization, the long-wave
 * limit of the Bloch problem (Sec. 5.1: the long-wave group velocity is the
 * speed of the equivalent homogeneous medium).  For each unit macro strain E_j
 * (Voigt order 11, 22, 33, 23, 13, 12, engineering shear) the periodic
 * fluctuation u solves K(0) u^ = i B(xi)^H F[C(x) E_j] by the preconditioned CG
 * of bw_pcg_solve (Sec. 3.3, Algorithm "InvA"); column j of the result is the
 * volume mean of C(x) (E_j + eps(u)) with eps(u) = F^-1[i B(xi) u^] (its real
 * part: on an even grid the Nyquist label -n/2 has no partner and the
 * fluctuation is not real).  rho_bar c^2 of bw_long_wave_speeds are the
 * Christoffel eigenvalues of this tensor up to the discretization's
 * even-grid offset.  rtol: relative residual of the six cell problems (0 ->
 * 1e-12 for BW_FP64, 1e-6 for BW_MIXED); maxit <= 0 -> 20000.  C66_host:
 * float64[36], row-major, symmetrized, Pa; iters_host: optional int32[6].
 * Returns BW_ENOTCONV (with C66_host filled) when a cell problem missed rtol.
 * Synchronizes `stream`. */
int bw_effective_stiffness(bw_rve* rve, double rtol, int32_t maxit, double* C66_host, int32_t* iters_host,
                           void* stream);

/* Diagnostics: a plain streaming copy of `bytes` (a multiple of 16, below
 * 2^39; 16-byte aligned device buffers, not overlapping) on `stream`, the
 * reference kernel for calibrating memory-traffic counters (its algorithmic
 * traffic is exactly `bytes` read and `bytes` written) and for the measured
 * device-copy bandwidth that kernel roofline fractions are also quoted
 * against. */
int bw_diag_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* Thread-local message describing the last non-zero status. */
const char* bw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BLOCHWAVE_H */
