/*
 * fockmi -- the HSE screened Fock-like exchange operator on an MI355X (gfx950).
 *
 * C ABI of the library libfockmi.so. Every entry point takes plain pointers
 * and sizes; device pointers are HIP device memory owned by the caller, the
 * stream argument is a hipStream_t passed as void* (NULL = the default
 * stream). No entry point frees caller memory. Status codes are returned;
 * nothing throws across the ABI; fock_last_error() gives a thread-local
 * message for the last failing call.
 *
 * Operation (Sato, Taniguchi, Shinohara, Yabana, Sec. II C "Nonlocal
 * Fock-like term", Eqs. (14)-(16); HSE composition Eq. (8)):
 *
 *   For orbitals given as periodic parts u_{jk}(r_m) on an n1 x n2 x n3 grid
 *   of the cell, normalised to (Omega/N_r) sum_m |u|^2 = 1, and target fields
 *   phi_{ik} at the same k-points,
 *
 *     W    = (1/N_r) IDFT( K_{k-k'} * DFT( conj(u_{jk'}) * phi_{ik} ) )
 *     (V_x phi)_{ik} = -(1/N_k) sum_{k', j} u_{jk'} * W
 *
 *   with the erfc-screened kernel K_q[l] = v(q + G_l),
 *     v(p) = 4 pi/|p|^2 (1 - exp(-|p|^2 / 4 w^2)),  v(0) = pi / w^2,
 *   q = k - k' never folded, G_l in FFT (fftfreq) order, and kernel entries
 *   on a Nyquist slot (l_d = -n_d/2) averaged over l_d = +-n_d/2.
 *   The exchange energy (E_xc piece of Eq. (22), closed shell) is
 *     E_x = (g_s/2)(1/N_k)(Omega/N_r) sum_{ik,m} conj(u_{ik}) (V_x u)_{ik}.
 *
 * Data layout of every orbital array: [k][band][m1][m2][m3], m3 fastest,
 * interleaved complex128 (re, im) in the cell's real-space grid, 16-byte
 * aligned. All k-points of a cell are present in every array.
 */
#ifndef FOCKMI_H
#define FOCKMI_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fockmi_plan_s* fockmi_plan;

typedef enum {
  FOCK_OK = 0,
  FOCK_WARN_NORM = 1,    /* taylor_step: norm drift above the plan threshold (psi still written) */
  FOCK_WARN_CONV = 2,    /* fock_eigensolve: maxit reached above tol (the current vectors still written) */
  FOCK_ERR_ARG = -1,     /* null / misaligned pointer, bad index, aliasing, bad scalar */
  FOCK_ERR_SIZE = -2,    /* grid length outside {16, 20, 24, 32}, or a form that needs a cubic grid */
  FOCK_ERR_HIP = -3,     /* a HIP runtime call failed (message in fock_last_error) */
  FOCK_ERR_NOMEM = -4,   /* device allocation failed or exceeded the plan's workspace cap */
  FOCK_ERR_STATE = -5    /* plan unusable (destroyed, or created on another device) */
} fock_status;

typedef enum {
  FOCK_FP64 = 0,         /* plain FP64 path: one stage per kernel through HBM */
  FOCK_FP32_COMP = 1,    /* fused pair kernel: complex64 pair FFTs; the sum over the bands j
                            of one k' in FP32 over at most 16 bands at a time, each such
                            partial sum added into an FP64 running sum with Neumaier
                            compensation, so the FP32 error does not grow with N_b.
                            Cells whose grid is not cubic run the plain stages with
                            complex64 pair products and FFTs and FP64 sums */
  FOCK_FP64_FUSED = 2    /* fused pair kernel in FP64 throughout (complex128 pair FFTs, one FP64
                            sum over all pairs) for cubic grids of length 16, 20 or 24; other
                            cells of such a plan run the plain FP64 stages */
} fock_prec;

typedef struct {
  int n[3];              /* FFT grid, each in {16, 20, 24, 32}; FOCK_FP32_COMP needs n1=n2=n3 */
  double a[3][3];        /* lattice vectors (bohr), one per row */
  int nk;                /* number of k-points (>= 1) */
  const double* kpts;    /* HOST [nk][3] Cartesian k-points (bohr^-1); copied at plan creation */
  int nb;                /* occupied bands per k-point (all fully occupied) */
  double omega;          /* screening parameter w (bohr^-1), > 0 */
  double gs;             /* spin degeneracy used by fock_energy (2 = closed shell) */
  /* Down-sampling (Sec. II C, after Eq. (16)): the sum over occupied orbitals
   * runs over the k-points of a sub-mesh S only, with weight 1/|S| in place
   * of 1/N_k (the paper samples 4^3 q-points for a 12^3 k-mesh). Every
   * orbital array still holds all nk k-points; u_occ enters only at S.
   * nsrc = 0 (or src = NULL) means S = every k-point. */
  int nsrc;              /* |S|, 0 <= nsrc <= nk */
  const int* src;        /* HOST [nsrc] distinct indices into kpts; copied at plan creation */
} fock_cell_desc;

/* Creates a plan for ncells cells on the current HIP device. Builds the kernel
 * tables K_q for every distinct q = k_i - k_j of each cell (FP64 on the GPU;
 * FP32 copies for FOCK_FP32_COMP). tune_cache_json may be NULL; otherwise it
 * is a path to the autotuner's JSON cache (read, and written after tuning).
 * Errors: FOCK_ERR_ARG (also for a source set with repeated or out-of-range
 * indices), FOCK_ERR_SIZE, FOCK_ERR_HIP, FOCK_ERR_NOMEM. */
fock_status fock_plan_create(const fock_cell_desc* cells, int ncells, fock_prec prec,
                             const char* tune_cache_json, fockmi_plan* out);

/* Frees everything the plan owns (never caller memory). NULL is accepted. */
fock_status fock_plan_destroy(fockmi_plan plan);

/* Eqs. (15)-(16): vphi[k][p] = (V_x[u_occ] phi)[k][p] for p < nphi, the sum
 * running over the source k-points S of the cell (all k unless down-sampled)
 * with weight 1/|S|.
 *   u_occ : device [nk][nb][N_r] complex128, occupied orbitals
 *   phi   : device [nk][nphi][N_r] complex128 target fields (may equal u_occ)
 *   vphi  : device [nk][nphi][N_r] complex128 output, overwritten; must not
 *           overlap u_occ or phi
 * nphi >= 1: an empty target set is FOCK_ERR_ARG, as are a NULL or misaligned
 * pointer, a cell index out of range and an output that overlaps an input;
 * nothing is launched then.
 * With phi == u_occ on a 32^3 cell of at least 3 k-points (FOCK_FP32_COMP,
 * no down-sampling) the pair kernel computes each pair of k-points once and
 * adds its conjugate term to the other target through per-XCD mirror copies:
 * the plan then holds 8 * nk * nb * N_r * 32 bytes of them (29 GB for
 * 216 k-points and 16 bands). The result is bitwise repeatable and agrees
 * with the form that runs every pair to rounding; that form runs instead
 * when the copies exceed the plan's workspace cap or the free device memory,
 * or with FOCKMI_SPLIT_SYM=0 at plan creation.
 * Stream-ordered; returns without synchronising. */
fock_status fock_apply(fockmi_plan plan, int cell, const void* u_occ, const void* phi, int nphi,
                       void* vphi, void* stream);

/* Eqs. (15)-(16) for a contiguous range of output k-points only: one GPU's
 * share when the output k-points are divided among GPUs (every GPU needs all
 * occupied orbitals as sources).
 *   vphi[k][p] = (V_x[u_occ] phi)[k0 + k][p] for k < nk_out, p < nphi
 *   u_occ : device [nk][nb][N_r] complex128, all occupied orbitals
 *   phi   : device [nk_out][nphi][N_r] complex128, the targets at k0 .. k0 + nk_out - 1
 *   vphi  : device [nk_out][nphi][N_r] complex128 output, overwritten; must not overlap
 *           u_occ or phi
 * 0 <= k0, nk_out >= 1, k0 + nk_out <= nk and nphi >= 1 (FOCK_ERR_ARG otherwise). Each target's sum is the
 * one fock_apply computes; the plain FP64 path and the grid forms of the fused
 * kernel give the same bits, the 32^3 lockstep form may group its FP64
 * additions differently, and fock_apply's pair-symmetric 32^3 form (phi ==
 * u_occ) adds each target's terms in another order (a k-range runs every
 * pair of its targets). Stream-ordered. */
fock_status fock_apply_krange(fockmi_plan plan, int cell, const void* u_occ, int k0, int nk_out, const void* phi,
                              int nphi, void* vphi, void* stream);

/* Exchange energy of u_occ (the E_xc piece of Eq. (22)) in FP64 (the final
 * reduction in double-double, rounded once):
 *   *ex_re, *ex_im <- E_x (the imaginary part is a check, zero in exact arithmetic).
 * Host pointers; synchronises the stream. Either output pointer may be NULL. */
fock_status fock_energy(fockmi_plan plan, int cell, const void* u_occ, double* ex_re, double* ex_im,
                        void* stream);

/* Reverse mode of fock_energy (derived from Eqs. (15)-(16) and the E_x piece of
 * Eq. (22)): for the cotangent g_e of E_x,
 *   g_u[k][j] <- g_e dE_x/du_{jk}   (PyTorch convention: dL/dRe + i dL/dIm)
 * With every k-point a source this is 4 w g_e (V_x[u] u)_{jk}, w = (g_s/2)(1/N_k)(Omega/N_r).
 * For a down-sampled cell it is 2 w g_e (V_x[u] u)_{jk} (u as the target) plus, at
 * the source k-points k' in S, the source-side adjoint
 *   -(2 w g_e/|S|) sum_{k,i} u_ik * W_{k'-k}(conj(u_ik) u_jk').
 *   u_occ : device [nk][nb][N_r] complex128;  g_u : device, same shape, overwritten,
 *           must not overlap u_occ.
 * Stream-ordered. FOCK_ERR_ARG for NULL/misaligned pointers or a non-finite g_e. */
fock_status fock_energy_vjp(fockmi_plan plan, int cell, const void* u_occ, double g_e, void* g_u_occ, void* stream);

/* Reverse mode of fock_apply (derived from Eq. (15)). Given the cotangent
 * g_vphi of vphi (PyTorch convention: dL/dRe + i dL/dIm), writes
 *   g_phi[k][p] = (V_x[u] g)[k][p]                       (device [nk][nphi][N_r], may be NULL)
 *   g_u[k'][j]  = -(1/|S|) sum_{k,i} ( g_ik * W_{k'-k}(conj(phi_ik) u_jk')
 *                                    + phi_ik * W_{k'-k}(conj(g_ik) u_jk') )   for k' in S,
 *                 0 for k' outside S                      (device [nk][nb][N_r], may be NULL)
 * Outputs are overwritten and must not overlap the inputs. Stream-ordered. */
fock_status fock_vjp(fockmi_plan plan, int cell, const void* u_occ, const void* phi, int nphi,
                     const void* g_vphi, void* g_u_occ, void* g_phi, void* stream);

/* One fourth-order Taylor step (Eqs. (9)-(10), with h(t+dt/2) ~ h(t)):
 *   psi <- sum_{m=0}^{order} (-i dt h)^m / m! psi,
 *   h = IDFT(|k+G+A/c|^2/2 DFT .) + v_loc + alpha * V_x[psi(t_n)]   (V_x frozen for the step)
 *   psi      : device [nk][nb][N_r] complex128, in place
 *   vloc     : device [N_r] float64 local potential, or NULL
 *   A_over_c : host [3] vector potential A(t_n)/c (bohr^-1)
 *   order    : 1..4 (4 is the paper's choice)
 *   max_norm_dev (host, may be NULL) <- max_{k,b} |(Omega/N_r)||psi_kb||^2 - 1| after the step
 * Synchronises the stream when max_norm_dev is requested. Returns FOCK_WARN_NORM
 * when that deviation exceeds 1e-6. */
fock_status taylor_step(fockmi_plan plan, int cell, void* psi, const double* vloc, const double A_over_c[3],
                        double dt, double alpha, int order, double* max_norm_dev, void* stream);

/* Predictor-corrector Taylor step (Sec. II C, Eqs. (11)-(13)) for the HSE functional:
 *   psi_pred = T(h(t)) psi          h(t) = T[A_now] + v_loc + alpha V_x[psi(t_n)]
 *   psi     <- T(h_c) psi           h_c  = T[A_mid] + v_loc + alpha (V_x[psi(t_n)] + V_x[psi_pred]) / 2
 * with T(h) = sum_{m=0}^{order} (-i dt h)^m / m!, the potentials at t + dt/2
 * taken as the averages of those at t and at t + dt (built from psi_pred), and
 * the external field at the midpoint exactly:
 *   A_now    : host [3] A(t_n)/c;   A_mid : host [3] A(t_n + dt/2)/c
 * Other arguments and the norm check as taylor_step. Three times the Fock
 * applications of taylor_step; second order in dt under a time-dependent field,
 * where taylor_step (A and V_x held at t_n) is first order. No reverse mode. */
fock_status taylor_step_pc(fockmi_plan plan, int cell, void* psi, const double* vloc, const double A_now[3],
                           const double A_mid[3], double dt, double alpha, int order, double* max_norm_dev,
                           void* stream);

/* Reverse mode of taylor_step for the same arguments (psi_n is the state
 * BEFORE the step); not available for a down-sampled cell (FOCK_ERR_ARG).
 * Given g_next, the cotangent of psi(t_n + dt):
 *   g_psi  : device [nk][nb][N_r] complex128 <- cotangent of psi(t_n), overwritten
 *   g_a    : host [3] <- d L / d (A/c) of this step (added to nothing; overwritten)
 * Stream-ordered, synchronises to return g_a. */
fock_status taylor_step_vjp(fockmi_plan plan, int cell, const void* psi_n, const double* vloc,
                            const double A_over_c[3], double dt, double alpha, int order,
                            const void* g_next, void* g_psi, double g_a[3], void* stream);

/* Energy functional of the propagated state (Eq. (22) restricted to the
 * pieces built here; E_GS is left to the caller); not available for a
 * down-sampled cell (FOCK_ERR_ARG):
 *   E = (g_s/N_k)(Omega/N_r) sum conj(psi) (T[A/c] + v_loc) psi + alpha * E_x[psi]
 *   *e_out    (host)   <- E
 *   grad_psi  (device [nk][nb][N_r] complex128, may be NULL) <- dE/dpsi in the
 *             PyTorch convention, 2 (g_s/N_k)(Omega/N_r) (T + v_loc + alpha V_x[psi]) psi
 *   grad_a    (host [3], may be NULL) <- dE/d(A/c) = (g_s/N_k)(Omega/N_r^2) sum_l (k+G_l+A/c) |DFT psi|^2
 * Synchronises the stream. */
fock_status taylor_energy(fockmi_plan plan, int cell, const void* psi, const double* vloc, const double A_over_c[3],
                          double alpha, double* e_out, void* grad_psi, double grad_a[3], void* stream);

/* Excitation energy of Eq. (22) with E_GS replaced by the energy of the initial
 * state (E_ex = E[psi_t; A_t/c] - E[psi_0; A_0/c], both as taylor_energy). Both
 * energies (about 86 Ha for the 24^3 / 64 k / 16-band differentiation workload)
 * are reduced in double-double and subtracted before the one final rounding, so
 * E_ex carries FP64 relative precision of its own instead of one unit in the last
 * place of E; central differences of E_ex at small steps rely on that.
 *   psi_t, psi_0 : device [nk][nb][N_r] complex128;  A_t, A_0 : host [3]
 *   *e_ex (host) <- E_ex.  Synchronises the stream. Not available for a down-sampled cell. */
fock_status taylor_excitation_energy(fockmi_plan plan, int cell, const void* psi_t, const double A_t[3],
                                     const void* psi_0, const double A_0[3], const double* vloc, double alpha,
                                     double* e_ex, void* stream);

/* Reverse mode of taylor_energy for the cotangent g_e of E (same arguments):
 *   g_psi (device, may be NULL) <- g_e dE/dpsi = 2 g_e (g_s/N_k)(Omega/N_r) (T + v_loc + alpha V_x[psi]) psi
 *   g_a   (host [3], may be NULL) <- g_e dE/d(A/c)
 * At least one output must be given. Synchronises the stream when g_a is requested. */
fock_status taylor_energy_vjp(fockmi_plan plan, int cell, const void* psi, const double* vloc,
                              const double A_over_c[3], double alpha, double g_e, void* g_psi, double g_a[3],
                              void* stream);

/* Macroscopic current of Eqs. (3)-(4) in the velocity gauge (no nonlocal
 * pseudopotential, electron charge -1):
 *   J = -(1/Omega)(g_s/N_k) sum_{k,b} int_cell Re[psi* (-i grad + A/c) psi] dr = -(1/Omega) dE/d(A/c)
 * (V_x does not depend on A in this gauge; only the kinetic term enters).
 *   psi : device [nk][nb][N_r] complex128;  A_over_c : host [3];  j_out : host [3] (a.u.)
 * Synchronises the stream. Not available for a down-sampled cell (FOCK_ERR_ARG). */
fock_status taylor_current(fockmi_plan plan, int cell, const void* psi, const double A_over_c[3], double j_out[3],
                           void* stream);

/* Modified Gram-Schmidt in band order, per k-point, in FP64 with the cell
 * inner product (Omega/N_r) sum conj(a) b (the normalisation that Eq. (15)
 * assumes for occupied orbitals). psi: device [nk][nb][N_r] complex128 in place. */
fock_status fock_orthonormalize(fockmi_plan plan, int cell, void* psi, void* stream);

/* Eigenstates of the Hamiltonian after the pulse (Sec. IV B, Eq. (25)): the nb
 * lowest eigenpairs, at every k, of
 *   h_k = IDFT(|k+G+A/c|^2/2 DFT .) + v_loc + alpha * V_x[u_occ]
 * (the propagator's h with the Fock-like term built from u_occ and held fixed),
 * by block LOBPCG in FP64 with a kinetic preconditioner.
 *   u_occ    : device [nk][nb][N_r] complex128, the orbitals that build V_x
 *   vloc     : device [N_r] float64 local potential, or NULL
 *   A_over_c : host [3] A/c (bohr^-1)
 *   phi      : device [nk][nb][N_r] complex128, in: a starting block of full rank
 *              (u_occ itself is a natural one), out: the eigenvectors in ascending
 *              order, (Omega/N_r) sum conj(phi_i) phi_j = delta_ij; must not alias u_occ
 *   tol      : stop when every residual (Omega/N_r)^(1/2) ||h phi - eps phi|| <= tol
 *   maxit    : iteration limit (each iteration applies h once to nb vectors per k)
 *   eig_host : host [nk][nb] <- eigenvalues (Ha), may be NULL
 *   res_host : host [nk][nb] <- final residual norms, may be NULL
 *   iters_host : host <- iterations taken, may be NULL
 * At most 16 bands per k (FOCK_ERR_SIZE otherwise). Synchronises the stream
 * once per iteration. Returns FOCK_WARN_CONV when maxit ends the iteration
 * above tol. The eigenvectors are unique up to phases where the eigenvalues
 * are; the span of all nb is unique when h has a gap above the nb-th. */
fock_status fock_eigensolve(fockmi_plan plan, int cell, const void* u_occ, const double* vloc,
                            const double A_over_c[3], double alpha, void* phi, double tol, int maxit,
                            double* eig_host, double* res_host, int* iters_host, void* stream);

/* Number density of excited electrons (Sec. IV B, Eq. (26)), with the k-point
 * sum written out:
 *   n_ex = (g_s / (N_k Omega)) sum_k [ nb - sum_{i,j} |<phi_ik | psi_jk>|^2 ],
 *   <a|b> = (Omega/N_r) sum_r conj(a) b,
 * phi the eigenvectors of fock_eigensolve (orthonormal), psi the time-dependent
 * orbitals, both device [nk][nb][N_r] complex128. *nex_host <- n_ex (bohr^-3).
 * FP64 with a fixed-order reduction; synchronises the stream. */
fock_status fock_excited_density(fockmi_plan plan, int cell, const void* phi, const void* psi, double* nex_host,
                                 void* stream);

/* All cells of the plan in one launch (FOCK_FP32_COMP plans with up to 8
 * cells of grid lengths 16, 20, 24, none down-sampled), replayed from a
 * captured hipGraph while the same buffers are passed: u_occ[c], phi[c],
 * vphi[c] as in fock_apply for cell c, nphi[c] targets. Host arrays of device
 * pointers, one entry per cell. The graph holds either one persistent kernel
 * over all cells or each cell's fused kernel on a stream of its own, forked
 * from the caller's stream (the default); a plan with a tuning cache measures
 * both on its first call. Other plans run their cells one after another.
 * Stream-ordered. */
fock_status fock_apply_batched(fockmi_plan plan, const void* const* u_occ, const void* const* phi,
                               const int* nphi, void* const* vphi, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): fock_apply
 * for a FOCK_FP32_COMP plan with the same arguments and result, which calls no
 * hipMalloc, hipFree or other allocating routine. Its scratch (the complex64
 * shadows of u_occ and phi, the Neumaier compensation field and, for 32^3 cells,
 * the FP32 band sums) comes from one fixed device array of 64 MiB that the
 * library holds on every GPU it runs on until the process ends. It runs the
 * grid form of the fused kernel (one workgroup per target), so for grid
 * lengths up to 24 it gives fock_apply's bits.
 * Errors: FOCK_ERR_SIZE when the cell needs more scratch than the fixed array
 * (about 32 MiB of shadows: e.g. 16^3 with up to ~500 orbitals) or its grid is
 * not cubic; FOCK_ERR_ARG as
 * fock_apply, and for a plan of another precision. Every call on one GPU uses
 * that GPU's one array: calls that overlap in time on one GPU (other streams,
 * other threads) race and must be serialised by the caller. Stream-ordered. */
fock_status fock_apply_noalloc(fockmi_plan plan, int cell, const void* u_occ, const void* phi, int nphi,
                               void* vphi, void* stream);

/* Diagnostics for measurement. While enabled, every launch of the fused pair
 * kernel (FOCK_FP32_COMP plans) and every batch of the plain path's pair
 * pipeline (FOCK_FP64 plans) is bracketed by HIP events recorded on the
 * caller's stream. fock_profile_read synchronises those events and returns
 * the summed elapsed time (ms) and the number of bracketed launches; reset=1
 * clears the record. Enabling costs two event records per launch. */
fock_status fock_profile_enable(fockmi_plan plan, int enable);
fock_status fock_profile_read(fockmi_plan plan, double* kernel_ms, long long* launches, int reset);

/* Diagnostics of the split 32^3 form of the FP32 fused kernel (one target on two
 * CUs of one XCD): the number of its launches, counted while profiling is
 * enabled, that stopped (a rendezvous timed out or the pair's CUs sat on two
 * XCDs) and whose result therefore came from the one-CU lockstep form launched
 * behind it. Synchronises the device; reset=1 clears the count. */
fock_status fock_profile_fallbacks(fockmi_plan plan, long long* count, int reset);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* fock_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
