/*
 * wpccc.h -- C ABI of the MI355X (gfx950) WP-CCC propagation library.
 *
 * The library integrates the close-coupling equations of the wave-packet
 * convergent-close-coupling method (arXiv:2403.04252, Eq. 1 and Eq. DIFFEQ)
 *
 *     dX/dz = M(z) X,   M = -(i/v) S(z)^{-1} H(z)
 *
 * along straight-line paths R = (b, 0, z) with the fourth-order Runge-Kutta
 * scheme of the paper's Algorithm 1, for a batch of impact parameters b at
 * once.  In the one-centre (1C) form S = I and H = D_T (Eq. NOINV, with the
 * -i/v of Eq. INV kept).  D_T is Eq. D1 with the radial integrals of Eq. D2
 * evaluated by the r-grid quadrature at the exact R = sqrt(b^2 + z^2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int status: WPCCC_OK (0) or a negative code.
 *    wpccc_last_error() returns a thread-local message for the last failure.
 *    No function aborts the process.
 *  - Handles (wpccc_basis_t, wpccc_plan_t) are owned by the library and are
 *    released with the matching *_destroy call.
 *  - Pointers named *_host are caller-owned host memory.  Pointers named
 *    *_dev are caller-owned device memory on the plan's device (for example
 *    a PyTorch tensor's data_ptr()).  The library never frees them.
 *  - Complex numbers are (re, im) pairs of doubles (HIP double2 layout).
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Device work is enqueued asynchronously on it.  Errors found on the
 *    device (non-finite amplitudes) are latched and returned by
 *    wpccc_plan_status(), which synchronises the stream.
 *  - There is no CPU path: without a usable gfx950 device, plan creation
 *    returns WPCCC_EHIP.
 *
 * State order (canonical, shared with every array below)
 * -------------------------------------------------------
 *  Radial functions are ordered by l, then bound states n = l+1..n_max, then
 *  wave-packet bins by increasing k.  States are ordered by l, then
 *  m = -l..l, then radial index: state (l, m, i) has index
 *  off_l + (m + l) * N_l + i with N_l = n_max - l + n_bins and
 *  off_l = sum_{l' < l} (2l'+1) N_l'.  State 0 is the ground state (1s),
 *  the paper's X[1] = 1 initial condition.
 */
#ifndef WPCCC_H
#define WPCCC_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define WPCCC_OK         0
#define WPCCC_EINVAL    -1   /* bad argument or specification */
#define WPCCC_ENOMEM    -2   /* host or device allocation failed */
#define WPCCC_EHIP      -3   /* a HIP runtime call failed (no device, launch error) */
#define WPCCC_ESINGULAR -4   /* exact zero pivot in an LU factorisation */
#define WPCCC_ENUMERIC  -5   /* non-finite amplitude detected on the device */
#define WPCCC_ENOTSUP   -6   /* requested form or size not supported by the library */

typedef struct wpccc_basis_s* wpccc_basis_t;
typedef struct wpccc_plan_s* wpccc_plan_t;

/* Message describing the last failure on the calling thread ("" if none). */
const char* wpccc_last_error(void);

/* Library version as "major.minor.patch". */
const char* wpccc_version(void);

/* ------------------------------------------------------------------------ */
/* Basis (Sec. II: bound eigenstates plus wave-packet pseudostates; the      */
/* r-grid of the paper's Sec. II, 0..r_max, denser near the origin).         */
/* ------------------------------------------------------------------------ */

/* Recipe of one centre's basis.
 *  n_max   bound hydrogen-like states n = 1..n_max with l <= min(n-1, l_max)
 *  l_max   largest orbital angular momentum (0..10)
 *  n_bins  wave-packet bins per l, uniform in k on [0, k_max] (0 = none)
 *  k_max   upper edge of the last bin (a.u.)
 *  n_r     number of grid intervals (even, 2..20000); r_i = r_max (i/n_r)^2
 *  r_max   grid extent (a.u.)
 *  Z       nuclear charge of the centre the states belong to (> 0)
 * Bound radial functions are the closed-form R_nl; a bin is
 * Delta_k^{-1/2} int_bin sqrt(2/pi) F_l(-Z/k, kr)/r dk (16-point
 * Gauss-Legendre per bin); per l the set is orthonormalised on the grid by
 * modified Gram-Schmidt (bound states first).  Energies: -Z^2/(2n^2) and
 * (k_lo^2 + k_lo k_hi + k_hi^2)/6. */
typedef struct {
    int n_max;
    int l_max;
    int n_bins;
    double k_max;
    int n_r;
    double r_max;
    double Z;
} wpccc_basis_spec;

/* Build a basis on the host (setup; not part of the propagation).
 * Errors: WPCCC_EINVAL for an invalid recipe, WPCCC_ENOMEM. */
int wpccc_basis(const wpccc_basis_spec* spec, wpccc_basis_t* out);

/* Sizes: number of states N, radial functions N_f and grid intervals n_r.
 * Any output pointer may be NULL. */
int wpccc_basis_info(wpccc_basis_t basis, int* n_states, int* n_radial, int* n_r);

/* Copy the basis out (host arrays, any may be NULL):
 *  r_host[n_r+1], w_host[n_r+1]      grid and Simpson weights
 *  phi_host[N_f*(n_r+1)]             radial functions, row-major [a][i]
 *  eps_host[N]                       state energies (a.u.)
 *  lmi_host[3*N]                     (l, m, radial index) per state */
int wpccc_basis_export(wpccc_basis_t basis, double* r_host, double* w_host,
                       double* phi_host, double* eps_host, int* lmi_host);

int wpccc_basis_destroy(wpccc_basis_t basis);

/* ------------------------------------------------------------------------ */
/* Plan: a batch of straight-line paths sharing one basis (1C).              */
/* ------------------------------------------------------------------------ */

/* lower-left block of H in the two-centre form */
#define WPCCC_Q_DAGGER 0   /* Q^dagger, as printed in Eq. 1 */
#define WPCCC_Q_PRIOR  1   /* <phi_P | -Z_P/r_P | phi_T>, the other side's potential; for a
                              set whose target and projectile are the same basis object it
                              is (-1)^(l_i + l_j) Q_ij by the symmetry of the quadrature
                              under exchange of the centres (not integrated again) */

typedef struct {
    double Zp;      /* 1C: projectile charge, the target electron sees -Zp/|r-R|
                       (Eq. D1 is written for Zp = 1; Zp = -1 is the negatively
                       charged projectile of Eq. NOINV).  0 means 1.  In 2C the
                       charges are the Z of the two bases. */
    int batched;    /* 1: all paths in each launch (default; 2C: the coupling
                       launches cover one basis-size group each, on a stream
                       per group, and each RK4 stage is one launch over the
                       paths of every group); 2 (2C): the stage launches per
                       group too; 0: one path per launch sequence, paths one
                       after another */
    int two_centre; /* set by wpccc_plan_create_2c; must be 0 for wpccc_plan_create */
    int q_lower;    /* 2C: WPCCC_Q_DAGGER (default) or WPCCC_Q_PRIOR */
    int n_eta;      /* 2C: Gauss-Laguerre nodes in eta (0 means 256) */
    int n_tau;      /* 2C: Gauss-Legendre nodes in tau (0 means 512) */
    double model_a; /* 1C: screened target potential V(r) = -(1 + a e^{-c r})/r on the */
    double model_c; /*     fixed basis: DeltaV = -a e^{-c r}/r is added to D_T (a = 0: none) */
    int checkpoint_every; /* wpccc_adjoint: steps between stored states (0: no
                             checkpoints, every state and stage input of the grid
                             kept, when they take at most 256 MiB; else ~sqrt(steps)) */
    int stage_rows; /* 1C: output rows per workgroup of the RK4 stage kernel, 4, 5,
                       6, 7, 8, 10, 12 or 16, with rows x (2 l_max + 1) <= 256
                       (WPCCC_EINVAL otherwise); 0: chosen at plan creation by
                       timing each admissible value on the plan's paths */
    int precision;  /* WPCCC_FP64 (default) or WPCCC_MIXED.  2C: overlap/transfer
                       contractions with FP32 products summed in FP32 over each
                       64-node chunk and in FP64 across chunks.  1C: the radial
                       moment tables of Eq. D2 stored in FP32 in scaled form,
                       (A_k / r_k^(lam+1), B_(k+1) r_(k+1)^lam), read at half the
                       bytes and combined with the R factors in FP64 (one
                       rounding per stored integral).  LU, solves, the angular
                       sums and RK4 stay FP64.  A 1C mixed plan runs one launch
                       per stage (WPCCC_ENOTSUP with WPCCC_LAUNCH_PERSISTENT)
                       and has no adjoint. */
    int graph;      /* 1C, batched: replay each 64-step chunk of wpccc_propagate
                       from a captured HIP graph (step lengths and positions
                       read from device memory); 2C: replay the steps of
                       wpccc_propagate from captured graphs, every group's
                       launches in one graph: with batched = 1 and
                       WPCCC_SOLVE_FACTORED each graph step runs the stages
                       of one step beside the couplings of the next (a step
                       whose start point z + h rounds away from the next
                       grid point begins a new run of graph steps);
                       otherwise one graph per start slot replays each step
                       whose start point the plan holds.  Both capture again when X moves; results
                       are bitwise those of launching kernel by kernel.
                       0: launch kernel by kernel */
    int stage_launch; /* 1C: how wpccc_propagate runs the RK4 stages of each
                       64-step chunk outside graph replays:
                       WPCCC_LAUNCH_AUTO (default): the faster of the two
                       forms below, timed at plan creation;
                       WPCCC_LAUNCH_STAGES: one launch per stage;
                       WPCCC_LAUNCH_PERSISTENT: one cooperative launch per
                       chunk whose workgroups stay resident and meet at a
                       per-path barrier between stages (WPCCC_ENOTSUP at plan
                       creation when its grid cannot be resident at once).
                       Both forms give bitwise the same amplitudes. */
    int radial;     /* 1C: how the radial integrals F of Eq. D2 are evaluated at R:
                       WPCCC_RADIAL_EXACT (default): the r-grid quadrature at the
                       exact R, from prefix/suffix moment tables;
                       WPCCC_RADIAL_INTERP: the paper's production form (Sec. II),
                       F tabulated on the r-grid nodes and interpolated at R by
                       the five-point Lagrange polynomial in r on the stencil of
                       the node nearest in sqrt(r / r_max), the multipole form
                       F(r_max) (r_max / R)^(lam+1) beyond the grid.  FP64, one
                       launch per stage (WPCCC_ENOTSUP with WPCCC_MIXED or
                       WPCCC_LAUNCH_PERSISTENT), no adjoint. */
    int stage_cache; /* 1C: WPCCC_CACHE_AUTO (default: timed at plan creation
                       where both forms apply), WPCCC_CACHE_ON or WPCCC_CACHE_OFF
                       (see wpccc_plan_stage_cache; WPCCC_ENOTSUP where the
                       form needs the cache) */
    int solve;      /* 2C: how each RK4 stage applies S^{-1} (Eq. INV):
                       WPCCC_SOLVE_FACTORED (default): S is factored once per
                       coupling point (LU with partial pivoting) and each
                       stage solves S y = H u with the two triangular factors;
                       WPCCC_SOLVE_EXPLICIT: the paper's form (Sec. II),
                       M = S^{-1} H formed once per coupling point from the
                       same factors with N right-hand sides, each stage the
                       product M u.  The same FP64 arithmetic up to the order
                       of the sums; the explicit form holds one more N x N
                       matrix per path and slot.  1C: must be 0. */
    int symmetric;  /* 2C: 1 replaces H by its S-norm-conserving form (not in the
                       paper; a variant of Eq. 1): H~ = (H + H^dag)/2 -
                       (i v / 2) dS/dz, which satisfies H~ - H~^dag = -i v dS/dz
                       so that X^dag S X is constant along the path.  dS/dz is
                       the central difference of S at z +- dz_sym, i.e. S at two
                       more positions per coupling point (three times the
                       coupling work).  FP64 and kernel-by-kernel only
                       (WPCCC_ENOTSUP with WPCCC_MIXED or graph).
                       wpccc_couplings returns H~.  1C: must be 0. */
    double dz_sym;  /* 2C symmetric: difference step in z (a.u.), 0 means 1e-4;
                       at most 0.01 */
} wpccc_plan_opts;

#define WPCCC_SOLVE_FACTORED 0
#define WPCCC_SOLVE_EXPLICIT 1

#define WPCCC_CACHE_AUTO 0
#define WPCCC_CACHE_ON   1
#define WPCCC_CACHE_OFF  2

#define WPCCC_RADIAL_EXACT  0
#define WPCCC_RADIAL_INTERP 1

#define WPCCC_LAUNCH_AUTO       0
#define WPCCC_LAUNCH_STAGES     1
#define WPCCC_LAUNCH_PERSISTENT 2

#define WPCCC_FP64  0
#define WPCCC_MIXED 1

/* Create a plan for n_traj paths with impact parameters b_host[j] > 0 and
 * speeds v_host[j] > 0 (a.u.), all expanded in `target`.  The basis must
 * outlive the plan.  Uploads the basis, builds the radial moment tables on
 * the device (synchronously on `stream`) and allocates the per-path
 * workspace.  opts may be NULL (defaults).
 * Errors: WPCCC_EINVAL, WPCCC_ENOMEM, WPCCC_EHIP, WPCCC_ENOTSUP (a basis
 * whose stage workgroup does not fit the LDS at any admissible tiling). */
int wpccc_plan_create(wpccc_basis_t target, int n_traj, const double* b_host,
                      const double* v_host, const wpccc_plan_opts* opts,
                      void* stream, wpccc_plan_t* out);

/* Two-centre plan (Eq. 1 with capture): n_sets pairs (targets[s],
 * projectiles[s]) of bases, path j expanded in pair set_of_traj[j] (bases of
 * uneven size may share one batch).  Each path has N_j = N_T + N_P states,
 * target states first, then projectile states, each in the canonical order.
 * Couplings: D_T (Eq. D1, charge Z of the projectile basis), D_P (Eq. D1
 * about the projectile, charge Z of the target basis), overlaps K and
 * transfer couplings Q by the spheroidal quadrature of Eq. K2 on n_eta x
 * n_tau nodes with the rotation of Eq. K1; M = -(i/v) S^{-1} H with S LU
 * factorised (partial pivoting) on the device.  The bases must outlive the
 * plan.  Errors: WPCCC_EINVAL, WPCCC_ENOMEM, WPCCC_EHIP. */
int wpccc_plan_create_2c(const wpccc_basis_t* targets, const wpccc_basis_t* projectiles,
                         int n_sets, int n_traj, const int* set_of_traj, const double* b_host,
                         const double* v_host, const wpccc_plan_opts* opts, void* stream,
                         wpccc_plan_t* out);

/* Size of path j's system: n_states = N_j, n_target = N_T of its set (equal
 * to N_j in 1C). */
int wpccc_plan_path_info(wpccc_plan_t plan, int j, int* n_states, int* n_target);

/* n_states: largest N_j of the plan; n_pad: row stride (in complex elements)
 * of the [n_traj][n_pad] amplitude arrays; device_bytes: device memory held. */
int wpccc_plan_info(wpccc_plan_t plan, int* n_traj, int* n_states, int* n_pad,
                    long long* device_bytes);

int wpccc_plan_destroy(wpccc_plan_t plan);

/* Rows per workgroup of a one-centre plan's RK4 stage kernel (stage_rows as
 * given, or as chosen by timing at plan creation). */
int wpccc_plan_stage_rows(wpccc_plan_t plan, int* rows);

/* Whether a one-centre plan's stage kernels take the radial integrals F from
 * a cache filled at the two new points of each step (1) or form them from the
 * moment table in every stage (0); chosen by timing at plan creation for the
 * exact-R forms (FP64 and WPCCC_MIXED), always 1 for the
 * WPCCC_RADIAL_INTERP form and for bases whose angular factors do not fit the
 * LDS; 0 for a two-centre plan.  In FP64 both give bitwise the same
 * amplitudes (in WPCCC_MIXED the cache holds F in FP32, one more rounding). */
int wpccc_plan_stage_cache(wpccc_plan_t plan, int* cached);

/* Launch form a one-centre plan's wpccc_propagate uses for its RK4 stages
 * (WPCCC_LAUNCH_STAGES or WPCCC_LAUNCH_PERSISTENT, as requested or as chosen
 * by timing at plan creation); WPCCC_LAUNCH_STAGES for a two-centre plan. */
int wpccc_plan_stage_launch(wpccc_plan_t plan, int* launch);

/* Returns the first device-side error latched since the last call (after
 * synchronising `stream`), then clears it: WPCCC_OK, WPCCC_ENUMERIC, (2C)
 * WPCCC_ESINGULAR with the path and pivot row in the message, or WPCCC_EHIP
 * when a barrier of the persistent stage kernel gave up waiting. */
int wpccc_plan_status(wpccc_plan_t plan, void* stream);

/* Couplings of path j at one z, with the interaction-picture phases
 * exp(i(eps_row - eps_col) z / v):
 *   H_dev  complex [N_j][N_j] row-major: 1C D_T(b_j, z) (Eq. D1/D2);
 *          2C [[D_T, Q], [Q^dagger or prior, D_P]] (Eq. 1)
 *   S_dev  2C: complex [N_j][N_j] row-major [[I, K], [K^dagger, I]];
 *          must be NULL in 1C.
 * Errors: WPCCC_EINVAL (j out of range, R = 0, S_dev NULL in 2C). */
int wpccc_couplings(wpccc_plan_t plan, int j, double z, void* H_dev, void* S_dev,
                    void* stream);

/* Allocation-free form of wpccc_couplings for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, output and errors as
 * wpccc_couplings for a one-centre plan; the per-point intermediates
 * (radial integrals, angular factors, phases) go to a fixed device array of
 * 8 MiB that the library holds on each GPU until the process ends (its
 * address is looked up once per device, on the first call there) instead of
 * the plan's workspace.  The call allocates nothing and calls no allocating
 * routine.  Every call on one GPU shares that array: calls that overlap in
 * time on one GPU (other streams or threads) race and must be serialised by
 * the caller.  Errors: as wpccc_couplings; WPCCC_ENOTSUP for a two-centre
 * plan or a basis whose intermediates exceed the 8 MiB. */
int wpccc_couplings_noalloc(wpccc_plan_t plan, int j, double z, void* H_dev, void* S_dev,
                            void* stream);

/* One RK4 step of Algorithm 1 from z to z + h for every path of the plan:
 * M is evaluated at z, z + h/2 and z + h.  X_dev: complex [n_traj][n_pad],
 * updated in place (entries beyond N are left untouched).
 * Errors: WPCCC_EINVAL (h == 0 or a path with R = 0 on the step). */
int wpccc_step(wpccc_plan_t plan, void* X_dev, double z, double h, void* stream);

/* Algorithm 1 over the whole z-grid zgrid_host[0..n_points-1] (strictly
 * increasing), starting from the amplitudes already in X_dev (set X = e_0
 * for the paper's initial condition).  M at each grid point is evaluated
 * once and carried to the next step, as in the paper.  On return (enqueued
 * on `stream`):
 *   X_dev     complex [n_traj][n_pad], amplitudes at zgrid[n_points-1]
 *   P_dev     double  [n_traj][n_pad], P_i = |X_i|^2 (may be NULL)
 *   norm_dev  double  [n_traj], X^dagger S X at the last point (1C: S = I;
 *             may be NULL)
 * Errors: WPCCC_EINVAL (fewer than 2 points, non-increasing grid);
 * WPCCC_ESINGULAR is latched (wpccc_plan_status) for an exact zero pivot. */
int wpccc_propagate(wpccc_plan_t plan, const double* zgrid_host, int n_points,
                    void* X_dev, void* P_dev, void* norm_dev, void* stream);

/* Gradients of a real loss of the final amplitudes (1C; Algorithm 1 on the
 * given grid differentiated exactly, reverse mode): the forward propagation
 * from X0 stores the state every `checkpoint_every` steps, the reverse sweep
 * recomputes each segment (keeping its states and RK4 stage inputs) and runs
 * the adjoint of every RK4 step,
 *   lambda_n = A_n^H lambda_(n+1),
 *   dL/dtheta += 2 Re(mu_k^H (dM/dtheta) u_k)  over the four stages,
 * with M^H = -M (Hermitian D_T) and dM/dtheta for theta = a, c (model
 * potential, plan options) and b (Eq. D1/D2 differentiated at fixed z).
 *   X0_dev    complex [n_traj][n_pad], initial amplitudes (read)
 *   X_dev     complex [n_traj][n_pad], final amplitudes (written; may be NULL)
 *   gX_dev    complex [n_traj][n_pad], dL/d conj(X) at the last point (read)
 *   grad_dev  double  [n_traj][3], per path dL/da, dL/dc, dL/db (written)
 * Device memory for the checkpoints is allocated by the first call.  Errors:
 * WPCCC_EINVAL (grid as wpccc_propagate), WPCCC_ENOTSUP (two-centre plan, a
 * WPCCC_MIXED or WPCCC_RADIAL_INTERP plan, or a basis whose operator kernel does not fit the LDS:
 * it takes 8 rows per workgroup, 4 where 8 do not fit, and 4, 2 or 1 with the
 * angular factors formed from the coefficient tables for the bases that need
 * the large-basis stage form; the paper's basis shape fits to l_max = 10). */
int wpccc_adjoint(wpccc_plan_t plan, const double* zgrid_host, int n_points, const void* X0_dev,
                  void* X_dev, const void* gX_dev, void* grad_dev, void* stream);

/* ------------------------------------------------------------------------ */
/* Observables at the end of the paths (Sec. II after Algorithm 1: the      */
/* final amplitudes give the cross sections of the reaction processes, from */
/* 30 to 50 paths per collision; Sec. III: the two-centre expansion         */
/* separates capture from ionisation).                                      */
/* ------------------------------------------------------------------------ */

/* Reaction channels, by the centre a state is expanded about and the sign
 * of its energy (bound eigenstates below zero, wave-packet pseudostates
 * above); index of each channel in the arrays below. */
#define WPCCC_N_CHANNELS       6
#define WPCCC_CH_ELASTIC       0   /* target state 0 (the initial state) */
#define WPCCC_CH_EXCITATION    1   /* other target states with eps < 0 */
#define WPCCC_CH_TARGET_CONT   2   /* target states with eps > 0 (ionisation, 1C: electron loss) */
#define WPCCC_CH_CAPTURE       3   /* projectile states with eps < 0 (2C) */
#define WPCCC_CH_PROJ_CONT     4   /* projectile states with eps > 0 (2C; ionisation with TARGET_CONT) */
#define WPCCC_CH_TOTAL         5   /* every state */

/* Groups of paths whose probabilities form one cross section: paths with the
 * same basis pair (set) and the same speed, numbered in order of first
 * appearance.  n_groups and group_of_traj_host[n_traj] may be NULL. */
int wpccc_plan_groups(wpccc_plan_t plan, int* n_groups, int* group_of_traj_host);

/* From the probabilities P_dev (double [n_traj][n_pad], as written by
 * wpccc_propagate):
 *   chan_dev   double [n_traj][WPCCC_N_CHANNELS]: the sum of P_i over the
 *              states of each channel (and over all states), per path
 *   sigma_dev  double [n_groups][WPCCC_N_CHANNELS] (may be NULL): the cross
 *              section of each channel per group, 2 pi int_0^inf P(b) b db by
 *              the trapezoidal rule over the group's impact parameters in
 *              increasing order (integrand 0 at b = 0, nothing added beyond
 *              the largest b), in a.u. (bohr^2)
 * Both are written on `stream`; sums are taken in a fixed order (the result
 * does not depend on scheduling).  Errors: WPCCC_EINVAL (NULL pointers). */
int wpccc_observables(wpccc_plan_t plan, const void* P_dev, void* chan_dev, void* sigma_dev, void* stream);

/* ------------------------------------------------------------------------ */
/* Diagnostics: per-kernel device time with HIP events; device ceilings.    */
/* ------------------------------------------------------------------------ */

/* enable != 0: from now on every kernel launch of this plan is bracketed by a
 * pair of HIP events recorded on the launch stream (adds a small gap between
 * launches); enable == 0 stops recording and drops collected records. */
int wpccc_plan_timing(wpccc_plan_t plan, int enable);

/* Synchronises the recorded events and returns the summed device time (ms)
 * and the number of launches of `kernel` ("k_stage", "k_slot_setup",
 * "k_couplings_dense", "k_probabilities", "k_moments") recorded since timing
 * was enabled or last read; the records are then cleared.
 * Errors: WPCCC_EINVAL (unknown kernel name). */
int wpccc_plan_kernel_time(wpccc_plan_t plan, const char* kernel, double* total_ms,
                           long long* launches);

/* Sustained matrix-core rates of the current device, measured with
 * back-to-back independent v_mfma_f64_16x16x4f64 (tflops_f64) and
 * v_mfma_f32_16x16x4f32 (tflops_f32) on every CU (four workgroups of four
 * waves each, eight accumulators per wave; about 40 ms on `stream`, which is
 * synchronised).  The ceiling the contraction kernels can reach, next to the
 * published peaks.  Either pointer may be NULL.  Errors: WPCCC_EHIP. */
int wpccc_measure_mfma(double* tflops_f64, double* tflops_f32, void* stream);

/* The linear solve of Sec. II (ZGESV with N right-hand sides, Eq. INV) for
 * caller matrices: X_b = A_b^{-1} B_b for b < batch, every A_b complex n x n
 * and B_b n x n (n right-hand sides), by the kernels the two-centre plans
 * use: LU with partial pivoting (largest |a|^2, ties to the lowest row),
 * then forward and backward substitution by 32 x 32 blocks.
 *  A_dev  complex128 [batch][n][n] column-major (A_b(i, j) at j*n + i), read only
 *  B_dev  complex128 [batch][n][n] row-major (B_b(i, k) at i*n + k), read only
 *  X_dev  complex128 [batch][n][n] row-major, written (may not alias A or B)
 * 1 <= n <= 2048.  Allocates its staging buffers and synchronises `stream`.
 * Errors: WPCCC_EINVAL (sizes, NULL), WPCCC_ENOMEM, WPCCC_EHIP,
 * WPCCC_ESINGULAR (an exactly zero pivot; the message names the first
 * such matrix and column; X then holds non-finite values). */
int wpccc_zgesv_batched(int n, int batch, const void* A_dev, const void* B_dev, void* X_dev, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* WPCCC_H */
