/*
 * pdz — perfect-hash (Paradeisos) Hubbard H.v and Lanczos on one MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only; no C++ types cross this boundary and
 * no exception escapes it.  Every function returns a pdz_status; on failure a
 * message is available from pdz_last_error() on the calling thread.
 *
 * Model (Sec. II.B, Eq. 1):
 *     H = - sum_{bonds (i,j)} t_ij sum_s (c+_{i,s} c_{j,s} + c+_{j,s} c_{i,s})
 *         + U sum_i n_{i,up} n_{i,dn}
 * on N sites with n_up up and n_dn down electrons (canonical ensemble,
 * Sec. II.A), dimension D = C(N, n_up) * C(N, n_dn).
 *
 * Basis and vector layout (Sec. II.A and Sec. III):
 *  - one spin species: site i <-> bit i of a uint32 occupation string; a
 *    sector lists every N-bit string with n set bits in ascending order;
 *  - a basis element is (phi_up, phi_dn), built from the vacuum with the up
 *    operators left of the down operators and the site index increasing from
 *    right to left;
 *  - its index is idx = C(N, n_dn) * idx_up(phi_up) + idx_dn(phi_dn), so a
 *    vector of length D is the row-major matrix X[idx_up][idx_dn];
 *  - idx_s(phi) is the forward map of Sec. III (Eq. 3): the sum over the set
 *    bits j_0 < j_1 < ... of C(j_m, m+1); its inverse is the backward map.
 *
 * Devices and streams: every call works on the HIP device current on the
 * calling thread.  `stream` is a hipStream_t (NULL = legacy default stream).
 * Device pointers must belong to that device.  Calls documented as
 * asynchronous only enqueue work on `stream`.
 *
 * Integer widths: sector ranks are uint32 (C(32,16) < 2^31); D, counts and
 * offsets are uint64.
 */
#ifndef PDZ_H
#define PDZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pdz_status;
#define PDZ_OK 0
#define PDZ_EINVAL (-1)   /* invalid argument (null pointer, bad bond, non-finite value, ...) */
#define PDZ_ERANGE (-2)   /* size outside the supported range */
#define PDZ_ENOMEM (-3)   /* device or host allocation failed */
#define PDZ_EHIP (-4)     /* a HIP runtime call failed */
#define PDZ_ENOCONV (-5)  /* iteration limit reached; results hold the best estimate */
#define PDZ_EDEVICE (-6)  /* a kernel found invalid device data (see pdz_device_errors) */

typedef enum { PDZ_F64 = 0, PDZ_F32 = 1 } pdz_dtype;

/* One undirected bond: contributes -t (c+_i c_j + c+_j c_i) for each spin
 * (Eq. 1).  i != j, 0 <= i, j < n_sites, t finite.  Repeated pairs add. */
typedef struct {
    int32_t i;
    int32_t j;
    double t;
} pdz_bond;

/* Opaque, immutable problem handle: sizes, tables and plans on one device. */
typedef struct pdz_problem_s* pdz_problem;

typedef struct {
    uint64_t D;          /* C(N,n_up) * C(N,n_dn)                          */
    uint64_t D_up;       /* C(N,n_up)                                       */
    uint64_t D_dn;       /* C(N,n_dn)                                       */
    uint64_t nnz;        /* structural nonzeros: D diagonal + all hops      */
    uint64_t hops_up;    /* allowed up hops summed over the up sector       */
    uint64_t hops_dn;    /* allowed down hops summed over the down sector   */
    int32_t n_sites, n_up, n_dn, n_bonds;
    int32_t max_hops_up; /* most hops out of one up-sector state            */
    int32_t max_hops_dn; /* most hops out of one down-sector state          */
    int32_t device;      /* HIP device the handle lives on                  */
    int32_t hv_path;     /* 0: sector hop tables, 1: on-the-fly ranks,
                            2: momentum space (D_up: every up string,
                            D_dn: every down string, hops_*: 0),
                            3: inversion parity (D: the subspace; D_up,
                            D_dn, hops_*: the real-space sectors; nnz:
                            an upper bound)                             */
} pdz_info;

/* ------------------------------------------------------------------ problems */

/* Validate the problem statement (Eq. 1; Sec. II.A), build the binomial table
 * C_i^m by Pascal's rule (Sec. III) and the per-sector hop tables on the
 * current device (each hop target ranked by the forward map on the device),
 * and return a handle.  Synchronous.
 * Errors: PDZ_ERANGE if n_sites < 1 or > 32 or D >= 2^62;
 *         PDZ_EINVAL for a null out/bonds (bonds may be NULL iff n_bonds == 0),
 *         n_bonds < 0, n_up/n_dn outside [0, n_sites], a bond with i == j or
 *         an endpoint outside [0, n_sites), a non-finite t or U;
 *         PDZ_ENOMEM / PDZ_EHIP from the device.
 * Ownership: the library owns everything behind the handle. */
pdz_status pdz_problem_create(int32_t n_sites, const pdz_bond* bonds, int32_t n_bonds, double U,
                              int32_t n_up, int32_t n_dn, pdz_problem* out);

/* Release a handle.  NULL is a no-op.  Synchronises the device first. */
pdz_status pdz_problem_destroy(pdz_problem p);

/* Sizes and counts of a problem (host only, no device work). */
pdz_status pdz_problem_info(pdz_problem p, pdz_info* out);

/* --------------------------------------------------------- the perfect hash */

/* Forward map (Sec. III, Eq. 3): ranks[k] = idx(bits[k]) within the sector of
 * N-bit strings with n set bits.  bits, ranks: device arrays of `count`
 * uint32.  A string whose popcount is not n, or with bits at or above
 * n_sites, gets rank 0xFFFFFFFF and raises the device error word.
 * Asynchronous.  Errors: PDZ_ERANGE (n_sites outside [1,32]), PDZ_EINVAL
 * (n outside [0,n_sites], null pointer with count > 0). */
pdz_status pdz_rank(int32_t n_sites, int32_t n, const uint32_t* bits, uint64_t count, uint32_t* ranks,
                    void* stream);

/* Backward map (Sec. III): bits[k] = the string of rank ranks[k].  A rank
 * >= C(n_sites, n) gives bits 0xFFFFFFFF and raises the device error word.
 * Asynchronous.  Errors as pdz_rank. */
pdz_status pdz_unrank(int32_t n_sites, int32_t n, const uint32_t* ranks, uint64_t count, uint32_t* bits,
                      void* stream);

/* Synchronise the current device, return the device error word raised by
 * kernels since the last call (0 if none) in *word, and clear it.
 * Returns PDZ_EDEVICE when the word was non-zero. */
pdz_status pdz_device_errors(uint32_t* word);

/* ------------------------------------------------------------------- H.v */

/* y = H x, matrix-free (Eq. 1), in precision dt (F64: doubles; F32: floats,
 * float accumulation).  x, y: device arrays of D elements in the layout above;
 * they must not overlap.  Each y element is summed by one thread in a fixed
 * order, so results are bitwise reproducible.  Asynchronous.
 * Errors: PDZ_EINVAL (null handle/pointer, overlapping x and y, bad dtype). */
pdz_status pdz_hv(pdz_problem p, pdz_dtype dt, const void* x, void* y, void* stream);

/* pdz_hv on vectors whose rows (one per up string) start `pitch` elements
 * apart: x and y hold D_up * pitch elements, element (u, d) at u * pitch + d;
 * columns D_dn..pitch-1 of x are not read and those of y are not written.
 * Same sums in the same order as pdz_hv, so the D elements are bitwise equal
 * to its output.  A pitch that is a multiple of 32 elements starts every row
 * on a 128-byte line, which the up pass reads faster (the layout pdz_lanczos
 * keeps its vectors in).  Real-space problems with hop tables only.
 * Errors: PDZ_EINVAL (as pdz_hv; pitch < D_dn; pitch != D_dn on a symmetry
 * sector or the on-the-fly path; pitch > 13,280 when the down pass that runs
 * is the scheduled one). */
pdz_status pdz_hv_pitched(pdz_problem p, pdz_dtype dt, const void* x, void* y, uint64_t pitch, void* stream);

/* ------------------------------------------------------ H.v launch plans */

/* Launch geometry of pdz_hv for one precision.  0 in a field = automatic.
 * down: looped family (summands of each element in hop-table order):
 *       1 one row per work group with the column's hop table loaded up front,
 *       2 one row with the table read in a loop, 3 two rows per work group,
 *       4 three rows per work group (1: 16-bit tables and at most 48 hops
 *       per state; 3, 4: the rows must fit in LDS);
 *       scheduled family (summands in the order of a gather schedule built
 *       at creation, in which the 32 lanes of a half-wave read 32 different
 *       LDS banks at every step): 5, 6, 7 one, two, three rows per work
 *       group (needs rows of 1024 to 13280 down states, at most two hop
 *       magnitudes; 6 and 7 F32 only);
 * up_cw: column-chunk width of the up-hop pass (F32: 32, 64, 128, 256;
 *       F64: 16, 32, 64, 128);
 * up: 1 the hops of a row are loaded in batches of 8, 2 all hops of a row are
 *       loaded before the first multiply-add (up_cw <= 64), 3 batches of 16
 *       (D < 2^32), 4 batches of 8 with 16-byte lanes, several rows of the
 *       chunk per wave (up_cw * element size <= 512 bytes; D < 2^32);
 * map: order of the up-pass tiles: 1 each XCD walks a pair of neighbouring
 *       column chunks at a time (blocks are dealt to XCDs round robin),
 *       2 chunk-major over all blocks, 3 each XCD walks one chunk at a time.
 * Plans of one down family compute the same y bit for bit.  Where the
 * scheduled family exists, the automatic plan and pdz_hv_tune use it alone,
 * so every plan they pick gives the same y; a looped variant set explicitly
 * differs from it by rounding only. */
typedef struct {
    int32_t down;
    int32_t up_cw;
    int32_t up;
    int32_t map;
} pdz_hv_plan;

typedef struct {
    pdz_hv_plan plan;
    double ms;           /* average duration of one pdz_hv with this plan */
} pdz_hv_trial;

/* Plan pdz_hv uses for precision dt (automatic fields resolved). */
pdz_status pdz_hv_get_plan(pdz_problem p, pdz_dtype dt, pdz_hv_plan* out);

/* Select a plan for precision dt.  The plan is the only mutable state of a
 * handle: do not call this while another thread launches pdz_hv on p.
 * Errors: PDZ_EINVAL for a plan this problem cannot run. */
pdz_status pdz_hv_set_plan(pdz_problem p, pdz_dtype dt, const pdz_hv_plan* plan);

/* Autotuner: time every valid plan for precision dt on the caller's device
 * buffers x, y (D elements each, not overlapping; x is read, y overwritten),
 * `reps` launches each after one warm-up launch, HIP events on `stream`;
 * select the fastest with pdz_hv_set_plan and return it in *best.  trials
 * (may be NULL) receives up to max_trials timings; *n_trials is the number of
 * plans timed, which may exceed max_trials.
 * Synchronous. */
pdz_status pdz_hv_tune(pdz_problem p, pdz_dtype dt, const void* x, void* y, int32_t reps, pdz_hv_trial* trials,
                       int32_t max_trials, int32_t* n_trials, pdz_hv_plan* best, void* stream);

/* Per-kernel profile of pdz_hv: after one warm-up, `reps` products y = H x
 * with a HIP event on `stream` before, between and after its two kernels,
 * then `reps` products back to back.  ms[0]: mean duration of the down pass
 * (diagonal and down-spin hops, writes y); ms[1]: of the up pass (up-spin
 * hops added onto y; 0 when the up sector has no hops); ms[2]: of one whole
 * pdz_hv in the back-to-back run.  A problem on the on-the-fly path has one
 * kernel: ms[0] is its duration, ms[1] = 0.  x, y as in pdz_hv (y = H x on
 * return).  reps in [1, 1000].  Synchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_hv_kernel_times(pdz_problem p, pdz_dtype dt, const void* x, void* y, int32_t reps, double* ms,
                               void* stream);

/* ---------------------------------------------------------------- Lanczos */

typedef struct {
    int32_t max_iter;      /* >= 1: Lanczos steps at most                                       */
    double tol;            /* accept when beta_{k+1} |s_k| <= tol * |theta| (>= 0)              */
    int32_t storage;       /* pdz_dtype of the Krylov vectors and of H.v                        */
    int32_t reorth;        /* 0: three-term recurrence only; 1: local re-orthogonalisation     */
                           /*    (w against v_{k-1} and v_k, classical Gram-Schmidt twice);   */
                           /*    2: full (against every earlier v_j, twice).  1 and 2 keep    */
                           /*    every Lanczos vector in the workspace (max_iter + 1 of D     */
                           /*    elements) and run without graphs                             */
    uint64_t seed;         /* start vector when v0 == NULL: SplitMix64 output r -> 2u-1         */
    int32_t check_every;   /* host reads the device convergence flag every this many steps (>=1) */
    int32_t use_graph;     /* 1: replay blocks of check_every steps as a captured HIP graph     */
    int32_t refine;        /* 1: build the Ritz vector and return its FP64 Rayleigh quotient;   */
                           /* 2: also, when its FP64 residual r is too large for that quotient */
                           /*    to be within 1e-8 (|r|^2 / gap > 1e-8 |E0|, gap = distance to */
                           /*    the second Ritz value of T_k), run FP64 Lanczos from the Ritz  */
                           /*    vector (tol max(tol, 1e-12), max_iter at least 300) and its    */
                           /*    refined energy is returned (and the status is that run's);   */
                           /*    the workspace then holds that FP64 run's workspace too        */
    int32_t keep_basis;    /* 1: keep every Lanczos vector in the workspace (max_iter + 1 of D   */
                           /*    elements, rows padded as described at pdz_lanczos) so that   */
                           /*    refine combines them in one pass instead of                   */
                           /*    regenerating them with a second run of H.v products           */
} pdz_lanczos_opts;

typedef struct {
    double E0;             /* lowest Ritz value of the tridiagonal T_k                          */
    double resid_est;      /* beta_{k+1} |s_k|                                                  */
    double E0_refined;     /* FP64 Rayleigh quotient of the Ritz vector (refine == 1), else E0  */
    double resid_refined;  /* FP64 |H y - E0_refined y| / |y| (refine == 1), else -1           */
    double seconds;        /* wall time of the call                                             */
    int32_t iters;         /* Lanczos steps taken                                               */
    int32_t converged;     /* 1 if the tolerance was met or the Krylov space became invariant   */
    int32_t restart_iters; /* steps of the FP64 restart (refine == 2 when it ran), else 0       */
} pdz_lanczos_result;

/* The refine == 2 decision of pdz_lanczos (host only, no device): given the
 * Lanczos coefficients of T_k (alpha[0..k), beta[0..k], beta[j] coupling
 * steps j-1 and j), the refined energy E and the FP64 residual norm resid of
 * the Ritz vector, *restart = 1 when resid^2 / gap > 1e-8 |E|, i.e. when the
 * residual does not bound E to 1e-8 and the FP64 restart must run.  gap is
 * (theta_next - theta_1) / 10, theta_next the lowest eigenvalue of T_k above
 * the cluster of Ritz values within 1e-8 max(1, |theta_1|) of theta_1 (ghost
 * copies or a degenerate level count once; the factor 10 allows for Ritz
 * values lying above the eigenvalues they approximate); with no Ritz value
 * above the cluster the gap is unknown and *restart = 1.  *gap receives the
 * estimate (0 when unknown).  Errors: PDZ_EINVAL (null pointer, k outside
 * [1, 2000]). */
pdz_status pdz_refine_decision(const double* alpha, const double* beta, int32_t k, double E, double resid,
                               int32_t* restart, double* gap);

/* Fill *o with defaults: max_iter 300, tol 1e-12, F64, no reorth, seed 1,
 * check_every 10, use_graph 1, refine 0, keep_basis 0. */
pdz_status pdz_lanczos_default_opts(pdz_lanczos_opts* o);

/* Timing of the Lanczos step of pdz_lanczos (measurement aid): the seeded
 * start vector, then `steps` steps (1 <= steps < max_iter, tol taken as 0)
 * launched on `stream` without a graph, with HIP events between the launch
 * groups of each step.  ms (5 doubles) receives mean milliseconds per step:
 * [0] the down pass (it also carries out the recurrence update when
 * *fused == 1), [1] the up pass, [2] the separate update kernel (0 when
 * fused), [3] the scalar kernels (alpha, beta, tridiagonal solve), [4] the
 * whole step.  ws as for pdz_lanczos with these options (reorth must be 0);
 * its contents are overwritten.  Synchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_lanczos_kernel_times(pdz_problem p, const pdz_lanczos_opts* o, void* ws, size_t ws_bytes,
                                    int32_t steps, double* ms, int32_t* fused, void* stream);

/* ------------------------------------------- dynamical correlations */

/* Fermion operator between sectors, for the Lanczos continued fraction of a
 * dynamical correlation function (the method Sec. I cites): y = c_{site,spin} x
 * (op 0: one electron of that spin removed) or y = c+_{site,spin} x (op 1: one
 * added).  x: D(src) elements in the layout of `src`; y: D(dst) elements of
 * `dst`, a problem on the same sites whose fillings differ from those of src
 * by exactly that electron (its bonds and U are not used here).  Each target
 * state has at most one source state: its string of that spin with the site
 * toggled, ranked by the forward map (Eq. 3).  Sign: the operator order of H
 * (Sec. II.A, up operators left of down operators, site index growing from
 * right to left): (-1)^(electrons of that spin above the site), times
 * (-1)^(n_up) for a down operator.  spin 0 = up, 1 = down.  x and y must not
 * overlap.  Asynchronous.  Errors: PDZ_EINVAL (null pointer, site or spin or
 * op out of range, dst not the neighbouring sector, overlap, other device). */
pdz_status pdz_fermion_op(pdz_problem src, pdz_problem dst, int32_t site, int32_t spin, int32_t op, pdz_dtype dt,
                          const void* x, void* y, void* stream);

/* After pdz_lanczos on `ws` (same options; refine >= 1 if a Ritz vector was
 * requested): the n = min(steps, max_n) recurrence coefficients alpha[0..n)
 * and beta[0..n] (beta[0] = 0, beta[k] for k >= 1 the norm of the k-th
 * residual; T_n has diagonal alpha and off-diagonal beta[1..n-1]), and the
 * norm of the start vector.  Host arrays of max_n and max_n + 1 doubles.
 * Synchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_lanczos_coefficients(pdz_problem p, const pdz_lanczos_opts* o, const void* ws, size_t ws_bytes,
                                    int32_t max_n, double* alpha, double* beta, double* norm0, int32_t* n_out);

/* Continued fraction of the resolvent <v0|(w - H)^{-1}|v0> from n Lanczos
 * coefficients started at v0 (norm2 = |v0|^2):
 *   g(w) = norm2 / (w - alpha[0] - beta[1]^2 / (w - alpha[1] - ... - beta[n-1]^2 / (w - alpha[n-1]))),
 * for the nw complex points w = w_re + i w_im; exact for the Krylov space of
 * dimension n.  Host arrays; no device work.  Errors: PDZ_EINVAL. */
pdz_status pdz_continued_fraction(const double* alpha, const double* beta, int32_t n, double norm2,
                                  const double* w_re, const double* w_im, int32_t nw, double* g_re, double* g_im);

/* Bytes of device workspace pdz_lanczos needs for these options. */
pdz_status pdz_lanczos_workspace_size(pdz_problem p, const pdz_lanczos_opts* o, size_t* bytes);

/* Lowest eigenvalue of H by Lanczos (cited in Sec. I), device resident:
 * H.v, dot products (FP64 accumulation), the alpha/beta recurrence and the
 * tridiagonal eigensolve (Sturm bisection, FP64) all run on the device; the
 * host reads one flag per block of check_every steps.
 * v0: device array of D elements in `storage` precision, or NULL for the
 *     seeded start vector; it is normalised internally (not modified).
 * ws: caller-owned device workspace of at least pdz_lanczos_workspace_size
 *     bytes, 256-byte aligned.  Inside it a real-space problem whose rows hold
 *     1024 or more down strings keeps its Lanczos vectors with the rows padded
 *     to a multiple of 32 elements (zeros past D_dn), so that every row starts
 *     on a 128-byte line; v0 and ritz_out are in the plain basis order.
 *     ritz_out: NULL, or a device array of D doubles that receives the
 *     normalised Ritz vector (of the FP64 restart when one ran); it forces
 *     refine >= 1, so size the workspace with refine >= 1.  Synchronous.
 * Errors: PDZ_EINVAL (bad options, null handle/result, ws too small, zero or
 * non-finite start vector); PDZ_ENOCONV when max_iter is reached (res holds
 * the best estimate). */
pdz_status pdz_lanczos(pdz_problem p, const pdz_lanczos_opts* o, const void* v0, void* ws, size_t ws_bytes,
                       double* ritz_out, pdz_lanczos_result* res, void* stream);

/* Copy the Ritz values theta_1..theta_n of the last pdz_lanczos run that
 * used this workspace with these options (n = min(max_n, steps taken)) into
 * host memory; *n_out receives n.  Synchronous.  Errors: PDZ_EINVAL (NULL
 * argument, ws too small). */
pdz_status pdz_lanczos_history(pdz_problem p, const pdz_lanczos_opts* o, const void* ws, size_t ws_bytes,
                               int32_t max_n, double* theta_host, int32_t* n_out);

/* ----------------------------------------- translation symmetry (momentum) */

/* Band energies of a translation-invariant hopping (Sec. IV.A): for an
 * L1 x L2 periodic cluster with sites s = x + L1*y and the bonds of Eq. 1,
 * eps[k] = -(1/N) sum_bonds t 2 cos(k . (r_j - r_i)) at the momentum
 * k = (2 pi/L1 (k mod L1), 2 pi/L2 (k div L1)), N = L1 L2 values (for the
 * square lattice with t and t': -2t(cos kx + cos ky) - 4t' cos kx cos ky).
 * Host only.  Errors: PDZ_ERANGE (N outside [1, 32]); PDZ_EINVAL (NULL, bad
 * bond, a bond list not invariant under the lattice translations). */
pdz_status pdz_kspace_band(int32_t L1, int32_t L2, const pdz_bond* bonds, int32_t n_bonds, double* eps);

/* Hubbard problem in momentum space restricted to total momentum K (Sec. IV.A,
 * Eq. 4): H = sum_{k,s} eps_k n_{k,s} + (U/N) sum_{k,k',q} c+_{k+q,up}
 * c+_{k'-q,dn} c_{k',dn} c_{k,up} on the states of n_up + n_dn electrons whose
 * orbital momenta sum to K (orbital i = momentum i as in pdz_kspace_band;
 * momenta add modulo the Brillouin zone).  eps: N host doubles.
 * Basis order and index: the spin-full k-space forward map of Sec. IV.A with
 * the extended counts C_i^m(k) (Eq. 5, reading i as the number of orbitals
 * 0..i-1) and Ct_i^m(k) (Eq. 7): states ordered by the up string, then the
 * down string, as integers; a vector is the ragged matrix X[up string][rank
 * of the down string among those of momentum K - K_up].  Signs: within one
 * spin, c+_a c_b gives (-1)^(electrons strictly between a and b) (the operator
 * order of Sec. II.A).  The returned handle works with pdz_problem_info,
 * pdz_hv, pdz_lanczos* and pdz_problem_destroy (no launch plans, batches or
 * fermion operators).  Synchronous: builds the down strings of every momentum
 * (backward map), their move table (forward map) and the row table on the
 * device and checks that the spin-full forward map lays the rows end to end.
 * Errors: PDZ_ERANGE (N outside [1, 32], empty sector, a row longer than 8192
 * down strings, counts beyond 32 bits); PDZ_EINVAL (NULL, fillings outside
 * [0, N], K outside [0, N), non-finite eps or U); PDZ_EDEVICE (a map left its
 * range: a library fault); PDZ_ENOMEM / PDZ_EHIP. */
pdz_status pdz_kspace_problem_create(int32_t L1, int32_t L2, const double* eps, double U, int32_t n_up,
                                     int32_t n_dn, int32_t K, pdz_problem* out);

/* Spin-full k-space forward map: idx[t] = index of (up[t], dn[t]) in the
 * sector of p.  Device arrays of count elements.  A pair with the wrong
 * fillings, bits beyond N or another total momentum gets idx = 2^64 - 1 and
 * sets bit 1 of the device error word (pdz_device_errors).  Asynchronous.
 * Errors: PDZ_EINVAL (NULL, not a momentum-space problem). */
pdz_status pdz_kspace_rank(pdz_problem p, const uint32_t* up, const uint32_t* dn, uint64_t count, uint64_t* idx,
                           void* stream);

/* Spin-full k-space backward map: (up[t], dn[t]) of index idx[t].  An index
 * >= D gives 0xFFFFFFFF in both and sets bit 2 of the device error word.
 * Device arrays.  Asynchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_kspace_unrank(pdz_problem p, const uint64_t* idx, uint64_t count, uint32_t* up, uint32_t* dn,
                             void* stream);

/* Shape of a momentum-space problem: cluster sides, K, longest row (down
 * strings of one momentum), number of non-empty rows, and the source-row
 * elements one pdz_hv stages (sum over target rows and momentum transfers q
 * of up moves x source row length: the vector elements the kernel reads
 * besides x and y themselves).  Any output may be NULL.
 * Errors: PDZ_EINVAL (NULL p, not a momentum-space problem). */
pdz_status pdz_kspace_info(pdz_problem p, int32_t* L1, int32_t* L2, int32_t* K, uint32_t* row_max, uint64_t* rows,
                           uint64_t* staged);

/* ----------------------------------------------- inversion symmetry (parity) */

/* Hubbard problem (Eq. 1, as pdz_problem_create) restricted to the subspace of
 * inversion parity `parity` (+1 or -1) (Sec. IV.B).  Inversion F sends site i
 * to N-1-i in every operator (a chain reversed; for an Lx x Ly cluster with
 * sites s = x + Lx*y, the point inversion through its centre); the bond list
 * must be symmetric under it.  On a basis state F reverses both strings and
 * multiplies by sigma = (-1)^(n_up(n_up-1)/2 + n_dn(n_dn-1)/2).
 * Basis and index (decision tree of Sec. IV.B, per string: pair (bit N-1-d,
 * bit d) of class A (0,1), B (0,0), C (1,1); representatives are A strings
 * and palindromes; tree index = the tree's forward map with the counts
 * S_i^m = C_{i-2}^{m-1} + S_{i-2}^m + S_{i-2}^{m-2}): rows are the up
 * representatives in tree order; a row of a non-palindromic up string holds
 * every down string in mirror pairs (each down representative in tree order
 * followed by its mirror image, pairs at even columns) and then the down
 * palindromes in tree order; a row of a palindromic one holds the down
 * representatives in tree order (down palindromes only when sigma = parity).
 * Basis vectors: (|r> + parity F|r>)/sqrt(2), or |r> when F|r> = parity |r>.
 * The handle works with pdz_problem_info, pdz_hv, pdz_lanczos* and
 * pdz_problem_destroy (no launch plans, batches or fermion operators).
 * Read at creation: PDZ_PARITY_UP_LANES = 16, 32 or 64 (default) lanes per
 * row in the up pass of H.v (its column slab is that times 4 in FP32, 2 in
 * FP64; any other value fails with PDZ_EINVAL); PDZ_PARITY_GATHER=1 serves
 * the non-palindromic rows with the one-pass kernel; PDZ_PARITY_WIDE_TABLE=1
 * keeps the down pass on 32-bit hop entries where 16-bit pairs would fit.
 * Synchronous.  Errors: as pdz_problem_create; PDZ_EINVAL (parity not +-1,
 * bonds not mirror symmetric); PDZ_ERANGE (sectors too large for the hop
 * tables, empty subspace); PDZ_EDEVICE (a tree map failed its bijection
 * check: a library fault). */
pdz_status pdz_parity_problem_create(int32_t n_sites, const pdz_bond* bonds, int32_t n_bonds, double U, int32_t n_up,
                                     int32_t n_dn, int32_t parity, pdz_problem* out);

/* Index of basis states given as (up, dn) strings (device arrays).  A pair
 * that is not a basis state (an image, wrong fillings, an excluded
 * self-mapped state) gets 2^64 - 1 and sets bit 1 of the device error word.
 * Asynchronous.  Errors: PDZ_EINVAL (NULL, not a parity problem). */
pdz_status pdz_parity_rank(pdz_problem p, const uint32_t* up, const uint32_t* dn, uint64_t count, uint64_t* idx,
                           void* stream);

/* Basis state (up, dn) of each index (device arrays); an index >= D gives
 * 0xFFFFFFFF in both and sets bit 2 of the device error word.  Asynchronous.
 * Errors: PDZ_EINVAL. */
pdz_status pdz_parity_unrank(pdz_problem p, const uint64_t* idx, uint64_t count, uint32_t* up, uint32_t* dn,
                             void* stream);

/* ---------------------------------------------------------------- batches */

/* Many independent problems (each the H of Eq. 1 on its own sites, bonds, U
 * and electron numbers) solved together.  Their vectors are packed into one
 * device array: problem i occupies elements [off_i, off_i + D_i), off_i a
 * multiple of 64, and the gaps between problems are ignored on input and left
 * untouched on output by pdz_batch_hv.  Within its slice each vector has the
 * single-problem layout (idx = C(N, n_dn) idx_up + idx_dn, Sec. III). */
typedef struct pdz_batch_s* pdz_batch;

/* Batched H.v launch plan (0 = default for that field). */
typedef struct {
    int32_t tile_elems;   /* about this many vector elements per tile: 1024, 2048, 4096 or 8192      */
    int32_t block;        /* threads per work group: 256, 512 or 1024                                */
    int32_t wgs_per_cu;   /* persistent work groups per compute unit, 1..8                           */
    int32_t order;        /* tile queue order: 1 largest problems first, 2 problem order             */
} pdz_batch_plan;

typedef struct {
    pdz_batch_plan plan;
    double ms;            /* mean time of one pdz_batch_hv with this plan */
} pdz_batch_trial;

/* Group n >= 1 problems created on the current device.  The problems must
 * outlive the batch and use sector hop tables (every sector of at most 2^24
 * states); one row of the down sector (C(N, n_dn) values in FP64) must fit the
 * 160 KiB of LDS of one work group.  Errors: PDZ_EINVAL (NULL argument,
 * problem on another device), PDZ_ERANGE (a problem without hop tables or
 * with too long rows), PDZ_EHIP. */
pdz_status pdz_batch_create(const pdz_problem* problems, int32_t n, pdz_batch* out);

/* Release the batch (not its problems).  NULL is a no-op.  Synchronises the device. */
pdz_status pdz_batch_destroy(pdz_batch b);

/* Host array of n + 1 element offsets: offsets[i] = start of problem i,
 * offsets[n] = length of the packed array. */
pdz_status pdz_batch_offsets(pdz_batch b, uint64_t* offsets);

/* y_i = H_i x_i for every problem i of the batch, in one persistent launch:
 * work groups take tiles (problem, group of rows) from a device queue, so the
 * uneven sizes balance across the chip.  x, y: packed device arrays
 * (offsets[n] elements of precision dt), not overlapping.  Each output is
 * summed in the same order as pdz_hv on its problem, so results are bitwise
 * identical to n single calls.  Asynchronous on `stream`; capturable in a
 * HIP graph.  Calls on one batch must not overlap (they share its queue
 * counter).  Errors: PDZ_EINVAL. */
pdz_status pdz_batch_hv(pdz_batch b, pdz_dtype dt, const void* x, void* y, void* stream);

pdz_status pdz_batch_get_plan(pdz_batch b, pdz_batch_plan* out);
/* Errors: PDZ_EINVAL for a plan outside the ranges above. */
pdz_status pdz_batch_set_plan(pdz_batch b, const pdz_batch_plan* plan);

/* Autotuner: time every plan of the search space on x, y (packed arrays as
 * in pdz_batch_hv; y is overwritten), `reps` launches each after a warm-up,
 * select the fastest and return it in *best.  trials (may be NULL) receives
 * up to max_trials timings, *n_trials their count.  Synchronous. */
pdz_status pdz_batch_tune(pdz_batch b, pdz_dtype dt, const void* x, void* y, int32_t reps, pdz_batch_trial* trials,
                          int32_t max_trials, int32_t* n_trials, pdz_batch_plan* best, void* stream);

/* Bytes of device workspace pdz_batch_lanczos needs for these options. */
pdz_status pdz_batch_lanczos_workspace_size(pdz_batch b, const pdz_lanczos_opts* o, size_t* bytes);

/* Lowest eigenvalue of every problem of the batch by the Lanczos recurrence
 * of pdz_lanczos, all problems in lockstep: one batched H.v per step, FP64
 * alpha, beta, Ritz value and convergence flag per problem on the device, and
 * a converged problem skipped by every later kernel.  With use_graph, blocks
 * of check_every steps (rounded up to a multiple of 3) are replayed as one
 * captured HIP graph.  Problem i starts from the seeded vector of seed + i
 * (the pdz_lanczos start vector of that seed), so its result equals a
 * pdz_lanczos run with that seed up to summation order.  reorth and
 * keep_basis must be 0.
 * refine = 1: after the run, every problem's Lanczos vectors are regenerated
 * bit for bit from its start vector and stored alpha, beta, its Ritz vector
 * is accumulated in FP64 and normalised, and E0_refined / resid_refined are
 * its FP64 Rayleigh quotient and residual (one batched FP64 H.v); the
 * workspace then includes two FP64 packed vectors.  ws: caller-owned device
 * workspace, 256-byte aligned.
 * results: host array of n entries.  Synchronous.
 * Errors: PDZ_EINVAL (bad options, workspace too small, non-finite scalar);
 * PDZ_ENOCONV when some problem reached max_iter (results still hold every
 * problem's best estimate). */
pdz_status pdz_batch_lanczos(pdz_batch b, const pdz_lanczos_opts* o, void* ws, size_t ws_bytes,
                             pdz_lanczos_result* results, void* stream);

/* ----------------------------------------------------------- learned start */

/* A small network proposes the Lanczos start vector; nothing of the paper's
 * method is learned, and a seeded random start (pdz_lanczos with v0 = NULL)
 * stays the fallback.  Network: 32 inputs x_i = 2 n_i - 1 (n_i the up
 * occupation of site i for i < 16, the down occupation of site i - 16
 * otherwise), two tanh layers of 128 units, 2 linear outputs: o_0 = ln|psi|,
 * o_1 = logit of P(psi > 0).  Parameters: one vector of pdz_mlp_param_count()
 * = 20,994 values in the order W1 (128 x 32, row = unit), b1 (128), W2
 * (128 x 128), b2 (128), W3 (2 x 128), b3 (2).  The caller owns an FP32
 * master copy and a BF16 copy (uint16 bit patterns, round to nearest even)
 * of it; the kernels read the BF16 copy and multiply on the BF16 matrix cores
 * with FP32 accumulation.  Occupations are passed as pairs of uint32 (up
 * bits, down bits), n pairs for n states. */
int32_t pdz_mlp_param_count(void);

/* Initialise params (device, FP32) and params_bf16 (device): weights uniform
 * in +-1/sqrt(fan_in) from SplitMix64(seed) output k for parameter k, biases
 * zero.  Synchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_mlp_init(float* params, uint16_t* params_bf16, uint64_t seed);

/* params_bf16 = BF16 rounding of params.  Asynchronous. */
pdz_status pdz_mlp_to_bf16(const float* params, uint16_t* params_bf16, void* stream);

/* out (n x 2 FP32, device) = network outputs for the n states in occ.  act:
 * NULL, or 768 n bytes (16-byte aligned) that receive the BF16 activations a
 * training step needs: h1 (n x 128), h1 transposed (128 x n), h2 (n x 128).
 * Asynchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_mlp_forward(const uint16_t* params_bf16, const uint32_t* occ, uint64_t n, float* out, void* act,
                           void* stream);

/* Bytes of device workspace pdz_mlp_loss and pdz_mlp_backward need for a batch of n. */
pdz_status pdz_mlp_workspace_size(uint64_t n, size_t* bytes);

/* Loss of a batch: target (n x 2 FP32) holds ln|psi| and the sign (+1/-1) of
 * each state; loss = (1/n) sum (o_0 - ln|psi|)^2 + softplus(o_1) - y o_1 with
 * y = 1 for a positive sign.  dout (n x 2) receives d loss / d out; *loss (one
 * device double) the loss.  Asynchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_mlp_loss(const float* out, const float* target, uint64_t n, float* dout, double* loss, void* ws,
                        size_t ws_bytes, void* stream);

/* grad (20,994 FP32, device) = d(sum dout . out)/d params for the batch whose
 * forward pass stored `act`.  n a multiple of 32, at most 2^24.  ws: 256-byte
 * aligned, pdz_mlp_workspace_size(n) bytes.  Products on the matrix cores;
 * per-slice partial sums reduced in a fixed order (deterministic).
 * Asynchronous.  Errors: PDZ_EINVAL, PDZ_ERANGE. */
pdz_status pdz_mlp_backward(const uint16_t* params_bf16, const uint32_t* occ, uint64_t n, const void* act,
                            const float* dout, float* grad, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (Kingma and Ba 2015, Algorithm 1; step counts from 1) on
 * `count` FP32 parameters with moments m, v; refreshes params_bf16.
 * Asynchronous.  Errors: PDZ_EINVAL (step < 1, betas outside [0, 1)). */
pdz_status pdz_adam_step(float* params, uint16_t* params_bf16, const float* grad, float* m, float* v, uint64_t count,
                         float lr, float beta1, float beta2, float eps, int32_t step, void* stream);

/* Bytes of device workspace of the |psi|^2 sampler of problem p (8 D + small). */
pdz_status pdz_sampler_workspace_size(pdz_problem p, size_t* bytes);

/* Prepare sampling from psi (D doubles, device, not all zero): integer weights
 * w_r = floor(2^32 psi_r^2 / max psi^2) and their inclusive prefix sums,
 * exact in any order.  Asynchronous. */
pdz_status pdz_sampler_prepare(pdz_problem p, const double* psi, void* ws, size_t ws_bytes, void* stream);

/* Draw `count` states with probability w_r / sum w: draw j takes SplitMix64
 * output first + j of `seed`, scales it to t = floor(z W / 2^64) and returns
 * the first r whose prefix sum exceeds t.  occ (count pairs) receives the
 * occupations, target (count x 2 FP32) ln|psi_r| and the sign of gauge *
 * psi_r (gauge = +1 or -1), idx (NULL or count uint32) the indices r.
 * Asynchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_sample(pdz_problem p, const double* psi, const void* ws, size_t ws_bytes, uint64_t seed, uint64_t first,
                      uint64_t count, double gauge, uint32_t* occ, float* target, uint32_t* idx, void* stream);

/* Learned start vector over the whole basis of p: v0[r] = s exp(min(o_0, 60))
 * with s = +1 if o_1 >= 0 else -1, for the state of index r (backward maps of
 * Sec. III on both spins).  v0: D elements of precision dt (device).  The
 * vector is not normalised (pdz_lanczos normalises its start vector).  N <= 16.
 * Asynchronous.  Errors: PDZ_EINVAL, PDZ_ERANGE (N > 16). */
pdz_status pdz_start_vector(pdz_problem p, const uint16_t* params_bf16, pdz_dtype dt, void* v0, void* stream);

/* *result = sum a_i b_i over n device elements of precision dt, products and
 * sums in FP64.  Synchronous.  Errors: PDZ_EINVAL. */
pdz_status pdz_dot(pdz_dtype dt, const void* a, const void* b, uint64_t n, double* result, void* stream);

/* pdz_dot for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and summation order as pdz_dot, with the 1024 partial sums held in
 * a fixed device array of the library (8 KiB per device, kept until the
 * process ends) instead of memory allocated per call, and the result written
 * to device memory.  result: one double in device memory, written
 * asynchronously on `stream` (bitwise equal to pdz_dot's result for the same
 * inputs).  n is not limited: the partial sums are 1024 whatever n is.
 * Calls that overlap on one device (different streams, no ordering between
 * them) race on the shared array; calls ordered on one stream do not.  Calls
 * no allocating routine.  Asynchronous.  Errors: PDZ_EINVAL (NULL argument,
 * dtype), PDZ_EDEVICE / PDZ_EHIP when the array's device address cannot be
 * obtained. */
pdz_status pdz_dot_noalloc(pdz_dtype dt, const void* a, const void* b, uint64_t n, double* result, void* stream);

/* ------------------------------------------------------------------ misc */

/* Message of the last failing call on this thread ("" if none).  Valid until
 * the next pdz call on the same thread. */
const char* pdz_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t pdz_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PDZ_H */
