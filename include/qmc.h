/*
 * qmc.h -- C ABI of the MI355X particle-by-particle VMC library.
 *
 * The library runs the hot path of real-space variational Monte Carlo as
 * the QMCPACK overview paper (arXiv:1802.06922) defines it: walkers are
 * independent Markov chains sampling |Psi_T|^2 (section "Variational Monte
 * Carlo"); each sweep moves every electron once, in order, with a Gaussian
 * proposal and the Metropolis acceptance (section "Trial Moves", equations
 * trans_prob_alle and accept_reject); Psi_T = D_up D_dn exp(J) (equation
 * eq:msdj with one determinant) with orbitals from a periodic tricubic
 * B-spline table (section "B-spline basis sets"), single-row inverse updates
 * (section "Multi-Determinant Slater-Jastrow Form") and one- and two-body
 * Jastrow factors (section "Jastrow factors"); the local energy is kinetic
 * plus Ewald-summed Coulomb terms (section "Hamiltonian", equation
 * vmc:electron_ham).
 *
 * Conventions for every call:
 *  - Returns a qmc_status; never aborts.  qmc_last_error() gives a message.
 *  - Host input arrays are read (and copied where kept) before the call
 *    returns; the caller keeps ownership.  Device state belongs to the
 *    library until qmc_destroy_system().  Output buffers belong to the caller.
 *  - All device work is issued on the stream given at creation (NULL = the
 *    default stream).  Calls that return host data synchronise that stream;
 *    asynchronous device errors surface at the next synchronising call.
 *  - One handle is driven by one host thread at a time; distinct handles may
 *    be used concurrently.  Results depend only on (desc, table, seed,
 *    walker count), never on other handles sharing the GPU.
 *  - Positions are in bohr, stored wrapped into the cubic cell [0, L)^3.
 *    Electrons 0..n_up-1 are spin up, n_up..n_up+n_dn-1 spin down.
 */
#ifndef QMC_H
#define QMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qmc_system_s* qmc_system;   /* opaque; owned by the library */

typedef enum {
    QMC_OK = 0,
    QMC_ERR_ARG = 1,       /* invalid argument or inconsistent sizes */
    QMC_ERR_OOM = 2,       /* device memory (or the caller's arena) exhausted */
    QMC_ERR_SINGULAR = 3,  /* a Slater matrix had a zero pivot */
    QMC_ERR_DEVICE = 4,    /* a HIP runtime error */
    QMC_ERR_STATE = 5,     /* call out of order (e.g. sweep before init_walkers) */
    QMC_ERR_NUMERIC = 6    /* a non-finite local energy was produced (written as NaN) */
} qmc_status;

typedef enum { QMC_FP64 = 0, QMC_MIXED = 1 } qmc_precision;
typedef enum { QMC_J_NONE = 0, QMC_J_PADE = 1, QMC_J_BSPLINE = 2 } qmc_jastrow_kind;
typedef enum { QMC_H_KINETIC = 0, QMC_H_COULOMB_EWALD = 1 } qmc_hamiltonian;

#define QMC_MAX_KNOTS 32     /* largest B-spline Jastrow M (free control points) */

/*
 * System description (section "Jastrow factors" for the radial functions;
 * section "Hamiltonian" for the ions).  Copied by qmc_create_system().
 *
 *  n_up, n_dn     electrons per spin (n_up >= 1, n_dn >= 0, n_up+n_dn <= 1024)
 *  L              cubic cell side (bohr)
 *  n_ions, ion_pos[3*n_ions], ion_Z[n_ions]   host arrays; may be 0/NULL
 *  precision      QMC_FP64: table, orbital values and inverse in FP64.
 *                 QMC_MIXED: FP32 table, values, ratios and inverse; FP64
 *                 positions, Jastrow, log-determinant and energy sums.
 *  delay_rank     1 (or 0) = Sherman-Morrison after every accepted move;
 *                 K = 4, 8, 16, 32 or 64 = delayed update (section "Multi-
 *                 Determinant Slater-Jastrow Form"): windows of K moves share
 *                 one inverse, ratios come from Y = V B0 by Schur complements
 *                 and accepted rows are applied by one rank-m product per window
 *  recompute_period  sweeps between full FP64 inverse rebuilds (0 = never)
 *  sigma          Gaussian proposal width (bohr); the transition probability
 *                 has no drift, so it cancels in the acceptance
 *  seed           key of the Philox4x32-10 streams; the numbers for electron
 *                 i of walker w in sweep s depend only on (seed, w, s, i)
 *  hamiltonian    QMC_H_KINETIC or QMC_H_COULOMB_EWALD
 *  j2_kind        two-body radial function, used for every electron pair:
 *                 PADE: j2_params = {a, b}, j2_n = 2, u = a r / (1 + b r),
 *                 no cutoff (minimum-image distance).
 *                 BSPLINE: j2_params = p_1..p_M (j2_n = M <= QMC_MAX_KNOTS),
 *                 cutoff j2_rcut, u(r) = sum_m p_m B3(r M / rcut - m) with
 *                 p_0 = p_2 - 2 (rcut / M) u'(0); u'(0) = j2_cusp_same for
 *                 equal spins and j2_cusp_opp for opposite spins.
 *  j1_kind        one-body (electron-ion) radial function, NONE or BSPLINE
 *                 (j1_params = p_1..p_M, j1_rcut, cusp j1_cusp)
 *  tie_guard      MIXED only: relative half-width of the band around each
 *                 acceptance threshold inside which the decision is re-taken
 *                 in FP64 (0 = library default 1e-3).  The library widens
 *                 each move's band by bounds on the FP32 rounding of its
 *                 ratio and on the error of the walker's FP32 inverse (its
 *                 measured residual I - A B), so that the mixed path takes
 *                 the decisions of FP64 arithmetic.
 *  arena, arena_bytes  optional caller-owned device memory (e.g. from the
 *                 PyTorch caching allocator).  If arena != NULL every device
 *                 buffer of the handle is carved from it and nothing is
 *                 allocated; size it with qmc_estimate_device_bytes().
 *  j3_gamma       three-body electron-electron-ion term (section "Jastrow
 *                 factors", the form of Drummond et al.), or NULL for none: for
 *                 electrons i, j and ion I with a = r_iI, b = r_jI, c = r_ij,
 *                 u = sum_{l,m<=j3_m_ei, n<=j3_m_ee} g_lmn a^l b^m c^n
 *                 (a - h)^3 (b - h)^3 while a, b < h = j3_rcut / 2 (else 0),
 *                 J3 = sum_I sum_{i<j} u.  Layout [2][m_ei+1][m_ei+1][m_ee+1],
 *                 equal-spin pairs first; g_lmn must equal g_mln; orders
 *                 0..3; 0 < j3_rcut <= L/2; needs ions.  Copied.
 *  move_kind      QMC_MOVE_PBYP (0): a sweep moves the electrons one at a
 *                 time (section "Trial Moves", particle by particle);
 *                 QMC_MOVE_ALL (1): a sweep is one all-electron move per
 *                 walker, every electron proposed from the same PROPOSE
 *                 counters, one uniform per walker (electron 0's ACCEPT
 *                 counter), accepted with min(1, |Psi(R')/Psi(R)|^2) from FP64
 *                 Gauss-Jordan determinants of both spin blocks at R' and the
 *                 full Jastrow change; a singular matrix at R' rejects.
 *                 delay_rank and recompute_period do not apply.
 *                 QMC_MOVE_ALL_DRIFT (2): all-electron moves drawn from the
 *                 drift-diffusion distribution (section "Trial Moves", eq.
 *                 trans_prob_alle with the wavefunction force F = 2 grad ln
 *                 Psi and lambda = 1/2): time step tau = sigma^2, every
 *                 electron proposed at r + tau grad ln|Psi| + sigma xi, the
 *                 acceptance (eq. accept_reject) including the ratio of the
 *                 transition probabilities T(R'->R)/T(R->R').  N <= 1024.
 *                 In mixed precision the velocities are built from FP64
 *                 gradient rows and the FP64 inverses of the Gauss-Jordan
 *                 eliminations (both kept beside the FP32 state), so every
 *                 quantity that decides a move is FP64; only the local
 *                 energies read the FP32 rows.
 *                 QMC_MOVE_PBYP_DRIFT (3): particle-by-particle sweeps whose
 *                 moves are drawn from the drift-diffusion distribution of one
 *                 electron (section "Trial Moves"): electron i, in index
 *                 order, proposes r_i + tau v + sigma xi with v = grad_i
 *                 ln|Psi| at the configuration the earlier moves of the sweep
 *                 left, and accepts with min(1, R^2 exp(2 dJ) T(r'->r) /
 *                 T(r->r')), the velocity at r' from the updated inverse
 *                 column B[:,k] / R; R = 0 rejects.  The orbital row at each
 *                 proposal is evaluated inside the sequential chain
 *                 (Sherman-Morrison updates; delay_rank does not apply,
 *                 recompute_period does).  FP64 only (ARG otherwise); the
 *                 spin block's chain must fit one workgroup's LDS (ARG).
 */
enum { QMC_MOVE_PBYP = 0, QMC_MOVE_ALL = 1, QMC_MOVE_ALL_DRIFT = 2, QMC_MOVE_PBYP_DRIFT = 3 };

typedef struct {
    int32_t n_up, n_dn;
    double L;
    int32_t n_ions;
    const double* ion_pos;
    const double* ion_Z;
    int32_t precision;
    int32_t delay_rank;
    int32_t recompute_period;
    double sigma;
    uint64_t seed;
    int32_t hamiltonian;
    int32_t j2_kind;
    const double* j2_params;
    int32_t j2_n;
    double j2_rcut;
    double j2_cusp_same;
    double j2_cusp_opp;
    int32_t j1_kind;
    const double* j1_params;
    int32_t j1_n;
    double j1_rcut;
    double j1_cusp;
    double tie_guard;
    void* arena;
    size_t arena_bytes;
    int32_t move_kind;
    int32_t j3_m_ei, j3_m_ee;
    double j3_rcut;
    const double* j3_gamma;
} qmc_system_desc;

/* Create a handle (section "Code structure": a system description -- cell,
 * particles, trial wavefunction, Hamiltonian, precision -- that every method
 * works on).  hip_stream: a hipStream_t (e.g. PyTorch's current stream) or NULL.  Uses the device current at the call.  Errors: ARG for
 * invalid sizes or parameters, DEVICE, OOM. */
qmc_status qmc_create_system(const qmc_system_desc* desc, void* hip_stream, qmc_system* out);

/* Upload the orbital table (section "B-spline basis sets": 64 coefficients
 * per orbital per evaluation).  Layout [gx][gy][gz][n_orb], C order, the
 * coefficient of knot (ix, iy, iz) multiplying the tensor product of uniform
 * cubic B-splines centred on that knot; the grid is periodic with spacing
 * L/gx, L/gy, L/gz.  dtype: 8 (double) or 4 (float).  coefs_on_device: 0 =
 * host pointer, 1 = device pointer.  The data are copied (converted to the
 * handle's precision).  Errors: ARG if n_orb != max(n_up, n_dn), a grid side
 * < 4, or dtype not 4/8; OOM; DEVICE. */
qmc_status qmc_load_spline_table(qmc_system s, int32_t gx, int32_t gy, int32_t gz, int32_t n_orb,
                                 const void* coefs, int32_t dtype, int32_t coefs_on_device);

/* Create n_walkers walkers (>= 1), the starting distribution of the
 * walkers of section "Variational Monte Carlo".  pos: host [n_walkers][N][3]
 * or NULL; NULL draws every electron uniform in the cell from the INIT stream
 * of its walker (no selection of the draws: an ill-conditioned start of a
 * MIXED system runs in FP64 until it is well conditioned, see
 * qmc_get_precision_stats).  Builds the Slater matrices, inverts them in FP64 (Gauss-Jordan
 * with partial pivoting) and resets the sweep counter to 0.  Errors: STATE
 * without a table; ARG; OOM; SINGULAR if any Slater matrix has a zero pivot
 * (the walkers are then unusable until re-initialised). */
qmc_status qmc_init_walkers(qmc_system s, int32_t n_walkers, const double* pos);

/* Run n_sweeps particle-by-particle sweeps of every walker (section "Trial
 * Moves": sequential single-electron moves; equation accept_reject).  Each
 * sweep proposes every electron once, in index order, and accepts with
 * probability min(1, R^2 exp(2 dJ)), R the determinant ratio and dJ the
 * Jastrow change.  With move_kind QMC_MOVE_ALL or QMC_MOVE_ALL_DRIFT a sweep
 * is instead one all-electron move per walker (see qmc_system_desc), an
 * accepted walker counting as N accepted electrons.  n_accepted_out (nullable; non-NULL
 * synchronises): total accepted electron moves over all walkers and these
 * sweeps.  Errors: STATE before init_walkers; DEVICE. */
qmc_status qmc_sweep(qmc_system s, int32_t n_sweeps, uint64_t* n_accepted_out);

/* Local energy of every walker at its current configuration (section
 * "Hamiltonian": E_L = sum_n Psi^-1 H_n Psi).  out[W][4] = (kinetic,
 * electron-electron, electron-ion, ion-ion) in hartree; the Coulomb parts
 * are Ewald sums with a uniform neutralising background where the charge
 * does not cancel, each independent of the Ewald splitting.  MIXED: the
 * kinetic part reads an inverse refined by one FP64 correction step
 * X = B + B (I - A B) against the FP64 Slater matrix A, and the chain goes on
 * from X (the FP32 updates' drift is squared away; decisions are unchanged,
 * see qmc_get_precision_stats); walkers in the FP64 fallback read their FP64
 * inverse with the orbitals evaluated in FP64.  out_on_device: 0 = host buffer
 * (synchronises), 1 = device buffer (asynchronous).
 * Errors: STATE; DEVICE; NUMERIC (host output only) if a value is not finite. */
qmc_status qmc_measure_local_energy(qmc_system s, double* out, int32_t out_on_device);

/* n_steps VMC steps, each one sweep (as qmc_sweep) followed by the local
 * energies (as qmc_measure_local_energy) of every walker, the collection
 * after each step that section "Hamiltonian" prescribes.  energies_dev: device
 * buffer [n_steps][W][4], step k's energies at offset k*W*4 (caller-owned).
 * Results are bit for bit those of n_steps (qmc_sweep(s, 1) +
 * qmc_measure_local_energy) calls.  Step k's measurement runs on a side stream
 * of the handle while step k+1's proposals are evaluated on the handle's stream
 * (they touch disjoint buffers), and step k+1's move chain waits for it; all
 * work completes in the handle's stream order (asynchronous).
 * Errors: ARG (negative n_steps, NULL buffer), STATE before init_walkers, DEVICE. */
qmc_status qmc_run_steps(qmc_system s, int32_t n_steps, double* energies_dev);

/* ---- Diffusion Monte Carlo (section "Diffusion Monte Carlo") ----------------
 * The handle's W walker slots hold the population (fixed capacity); a slot is
 * alive while its weight is positive.  Needs move_kind QMC_MOVE_ALL_DRIFT or
 * QMC_MOVE_PBYP_DRIFT (then a step moves every electron of a slot once, a move
 * with R < 0 being rejected; the node-crossing count is per electron move).
 * A step: every slot makes one drift-diffusion all-electron move (section
 * "Trial Moves"), a move across a node of Psi being rejected (fixed node);
 * alive slots take w <- w exp(-tau (E_L(R) + E_L(R_new) - 2 E_T) / 2), tau =
 * sigma^2 (eqs. pmc:g_growth, pmc:walker_weight); the estimate is E = sum w
 * E_L / sum w (eq. pmc:weighted_average); branching gives each alive slot
 * M = INT(w + xi) copies (xi from the BRANCH counter of (slot, step)): M = 0
 * dies, M >= 1 keeps its slot and its M - 1 extra copies fill the free slots in
 * ascending order, lower slots' copies first (copies beyond the free slots are
 * dropped and counted); every walker alive afterwards has weight 1; then
 * E_T <- E - feedback ln(population / n_target).  Dead slots move too (their
 * results are never read), so a step runs entirely on the device. */

/* Start a population (section "Diffusion Monte Carlo": walkers of unit
 * weight drawn from the trial wavefunction's distribution, E_T near the
 * estimate): slots [0, n_target) alive with weight 1 at their current
 * configurations, local energies measured; E_T = e_trial, or (NaN) the mean
 * local energy of the alive slots; feedback >= 0 in hartree.  Synchronises.
 * The first call after qmc_init_walkers allocates the population buffers
 * (about 60 bytes per slot; qmc_estimate_device_bytes counts them).
 * Errors: STATE (no walkers, or no drift moves), ARG, OOM, NUMERIC. */
qmc_status qmc_dmc_init(qmc_system s, int32_t n_target, double e_trial, double feedback);

/* n_steps DMC steps on the handle's stream, asynchronous (section "Diffusion
 * Monte Carlo"; one step as described above, eqs. pmc:g_growth,
 * pmc:walker_weight, pmc:weighted_average).  stats_dev: device
 * buffer [n_steps][6] (caller-owned) receiving per step (E, sum of weights
 * before branching, population after branching, E_T used by the step, dropped
 * copies, moves rejected for crossing a node).  Errors: STATE, ARG, DEVICE. */
qmc_status qmc_dmc_steps(qmc_system s, int32_t n_steps, double* stats_dev);

/* Population state (section "Diffusion Monte Carlo", the walker weights of eq.
 * pmc:walker_weight after branching), host buffers, each nullable: weights[W] (0 = dead slot),
 * energies[W] (local energy of each slot's configuration), the current E_T and
 * the population.  Synchronises.  Errors: STATE; NUMERIC if the population died
 * out (the state is still returned). */
qmc_status qmc_dmc_get(qmc_system s, double* weights, double* energies, double* e_trial, int32_t* population);

/* Branching of the last DMC step (section "Diffusion Monte Carlo", eqs. pmc:g_growth and
 * pmc:walker_weight, then M = INT(w + xi)), host buffers [W] each, nullable:
 * weights = w G_B of every slot alive when the step began (0 for the others);
 * energies = the local energy of its new configuration (NaN for the others);
 * mult = its multiplicity M (0 for the others); plan = the slot whose walker was
 * copied into this slot (-1: none).  Free slots (M = 0) take the extra copies
 * (M - 1 of every slot, lower source slots first) in ascending order.  Synchronises.
 * Errors: STATE before qmc_dmc_init or before the first step. */
qmc_status qmc_dmc_get_branching(qmc_system s, double* weights, double* energies, int32_t* mult, int32_t* plan);

/* Walker state (section "Code structure": walkers persist between steps), copied
 * to host buffers (each nullable): pos[W][N][3];
 * logabs_det[W][2] = log|D_up|, log|D_dn| accumulated as the sum of
 * log|R| of the accepted moves since the last full inverse; sign[W][2]. */
qmc_status qmc_get_walkers(qmc_system s, double* pos, double* logabs_det, int32_t* sign);

/* Accept flags of the last sweep (eq. accept_reject per move), host [W][N],
 * 1 = accepted. */
qmc_status qmc_get_accept_log(qmc_system s, uint8_t* bits);

/* Counters (each nullable; section "Code structure", precision as a parameter
 * of the same algorithm): redecided = moves since qmc_init_walkers whose
 * acceptance fell inside the mixed-precision guard band and was decided again
 * from an FP64 ratio; sweeps = the index of the next sweep in the random
 * streams (the sweeps run since qmc_init_walkers, plus the index a resume set).
 * Synchronises. */
qmc_status qmc_get_counters(qmc_system s, uint64_t* redecided, uint64_t* sweeps);

/* Resume a saved run (section "Variational Monte Carlo": each walker is an
 * independent Markov chain; here its random numbers are counter-based draws
 * indexed by walker, sweep and electron).  After qmc_init_walkers with the saved
 * positions (qmc_get_walkers) this sets the index of the next sweep to the saved
 * one (qmc_get_counters), so the run continues on the same streams: the moves
 * propose what the uninterrupted run proposes and take its decisions (the
 * inverses are fresh eliminations of the same positions, so the ratios differ
 * only in rounding), and the periodic rebuild keeps its schedule (sweeps whose
 * index is a multiple of recompute_period).  A DMC population is not resumed.
 * Synchronises.  Errors: STATE before qmc_init_walkers; ARG for an index of
 * 2^32 or more. */
qmc_status qmc_set_sweep_index(qmc_system s, uint64_t sweep_index);

/* Mixed precision, particle-by-particle moves (section "Code structure": single, double and
 * mixed precision from one source): how the FP32 path keeps the FP64 decisions.
 * Every walker's inverse error ||I - A B||_F is measured after each full rebuild and by
 * the refinement before each measurement (A the FP64 Slater matrix); it widens that
 * walker's re-decision band (see tie_guard).  A walker whose measured error passes 2e-3 is
 * rebuilt in FP64 on its own; one whose freshly rounded FP32 inverse still errs by more
 * than 2e-4 (an ill-conditioned Slater matrix) runs its moves and its kinetic energy in
 * FP64 (fallback) until the error of its FP32 rounding drops below 5e-5.  Counters since
 * qmc_init_walkers (each nullable): early_rebuilds = single-walker FP64 rebuilds;
 * fallback_sweeps = walker sweeps run in FP64; fallback_now = walkers in fallback now;
 * fallback_mask = host [W], 1 for those walkers.  Zero for other systems.  Synchronises. */
qmc_status qmc_get_precision_stats(qmc_system s, uint64_t* early_rebuilds, uint64_t* fallback_sweeps,
                                   int32_t* fallback_now, int32_t* fallback_mask);

/* Rebuild every inverse from scratch in FP64 and reset log|D| (section
 * "Multi-Determinant Slater-Jastrow Form": the updated inverse is periodically
 * recomputed to bound the accumulated rounding).  drift_out (nullable, host
 * [W][2]): accumulated log|D| minus the rebuilt one. */
qmc_status qmc_recompute(qmc_system s, double* drift_out);

/* Diagnostic: value, gradient (x, y, z) and Laplacian of every orbital at n
 * host positions pos[n][3] (section "B-spline basis sets": 64 coefficients per
 * orbital and point), written to host out[n][5][n_orb] in FP64. */
qmc_status qmc_eval_spo_vgl(qmc_system s, int32_t n, const double* pos, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): qmc_eval_spo_vgl with
 * its device staging (the positions and the results) in one fixed array of
 * QMC_NOALLOC_DOUBLES doubles (4 MiB) per GPU, which the library holds until the
 * process ends, instead of two allocations per call; same arguments, same
 * results.  Needs n (3 + 5 n_orb) <= QMC_NOALLOC_DOUBLES (else QMC_ERR_ARG, with
 * nothing done).  Calls that overlap on one GPU race: they share the array.
 * Synchronises the handle's stream.  Errors: as qmc_eval_spo_vgl. */
#define QMC_NOALLOC_DOUBLES (1 << 19)
qmc_status qmc_eval_spo_vgl_noalloc(qmc_system s, int32_t n, const double* pos, double* out);

/* Kernel timing (section "Performance and Parallel Scaling": the time of each
 * part of a step): when enabled, every launch of each kernel class is
 * bracketed by HIP events on the handle's stream.  Classes: 0 = orbital
 * gather (proposal + spline VGL), 1 = move chain (ratio, Jastrow, accept,
 * inverse update), 2 = measurement (kinetic + Ewald), 3 = inverse rebuild.
 * qmc_kernel_timing synchronises and returns the summed milliseconds and the
 * launch count since the last reset (reset = 1 clears them). */
qmc_status qmc_set_timing(qmc_system s, int32_t enable);
qmc_status qmc_kernel_timing(qmc_system s, int32_t kernel_class, double* total_ms, int64_t* launches,
                             int32_t reset);

/* Change the delay rank between sweeps (1, or 4..64 a power of two; section
 * "Performance and Parallel Scaling", the delayed update).  Windows never span
 * sweeps, so any rank is valid at a sweep boundary. */
qmc_status qmc_set_delay_rank(qmc_system s, int32_t delay_rank);

/* Gather autotuner: times the orbital gather (section "B-spline basis sets")
 * with 1/4, 1/2, 1, 2 and 4 times the default number of lanes per proposal (lanes
 * split a proposal's orbitals, never a sum, so every width gives the same
 * rows bit for bit), trial_sweeps (>= 2; the first untimed) ordinary sweeps
 * each, and keeps the fastest for later sweeps and batches.  best_lanes_log2,
 * best_ms (nullable): the chosen width (log2 lanes) and its mean gather
 * milliseconds.  Errors: STATE before init_walkers or without a table. */
qmc_status qmc_autotune_gather(qmc_system s, int32_t trial_sweeps, int32_t* best_lanes_log2, double* best_ms);

/* Set the gather's lanes per proposal directly (section "B-spline basis sets":
 * the orbital evaluation's work split): lanes_log2 in 0..6, or -1 for the
 * default of the orbital count.  Errors: ARG outside that range. */
qmc_status qmc_set_gather_lanes(qmc_system s, int32_t lanes_log2);

/* Autotuner (section "Performance and Parallel Scaling": the delay rank is a
 * tunable of the delayed update): runs trial_sweeps sweeps (>= 2; the first is
 * not timed) with each candidate delay rank, times the move-chain kernel with HIP events, keeps the
 * fastest and writes it to best_rank (best_ms: its mean chain milliseconds per
 * sweep; both nullable).  The trial sweeps are ordinary sweeps of the chain. */
qmc_status qmc_autotune_delay(qmc_system s, const int32_t* ranks, int32_t n_ranks, int32_t trial_sweeps,
                              int32_t* best_rank, double* best_ms);

/* Local energies of the last measurement (section "Hamiltonian";
 * qmc_measure_local_energy or a batch sweep with measurement), host out[W][4].
 * Synchronises. */
qmc_status qmc_get_last_energies(qmc_system s, double* out);

/* ---- Batches: several systems advanced by fused launches -------------------
 * (Section "Adapting to trends in High Performance Computing": enough
 * independent work per launch to fill an accelerator.)
 * The walkers of all systems of a batch (any sizes, one precision, delay rank
 * >= 4, particle-by-particle moves, initialised) are advanced by one orbital-gather launch, one delayed-
 * chain launch per LDS class and one measurement launch per sweep.  Each
 * system's results are identical to advancing it alone.  All launches go to
 * the batch's stream.  qmc_batch_sweep orders itself after work already
 * queued on the members' own streams and orders later work on those streams
 * after itself (stream events), so member calls such as qmc_get_accept_log
 * may follow on the member's stream.  The batch does not own the systems;
 * re-create it after re-initialising or destroying a member. */
typedef struct qmc_batch_s* qmc_batch;

qmc_status qmc_batch_create(const qmc_system* systems, int32_t n_systems, void* hip_stream, qmc_batch* out);

/* n_sweeps sweeps (section "Trial Moves") of every member; measure != 0 also measures every member's
 * local energies after each sweep (read them with qmc_get_last_energies).
 * Member systems' periodic FP64 rebuilds run between sweeps as configured. */
qmc_status qmc_batch_sweep(qmc_batch b, int32_t n_sweeps, int32_t measure);

/* use_graph != 0: capture one sweep (all its launches) as a HIP graph on first
 * use and replay it for every later sweep (section "Adapting to trends in High
 * Performance Computing": launch overheads of small kernels). */
qmc_status qmc_batch_set_graph(qmc_batch b, int32_t use_graph);

/* Summed milliseconds and count of batch sweeps (HIP events around each
 * sweep, including its measurement; section "Performance and Parallel
 * Scaling") since the last reset; synchronises. */
qmc_status qmc_batch_timing(qmc_batch b, double* total_ms, int64_t* sweeps, int32_t reset);

/* Free the batch (section "Code structure": the members stay the caller's). */
qmc_status qmc_batch_destroy(qmc_batch b);

/* Free every device buffer of the handle and the handle itself (section "Code
 * structure": the handle owns the walkers' device state). */
qmc_status qmc_destroy_system(qmc_system s);

/* Message of the last error of s (NULL: of the last failed call on this
 * thread; section "Code structure", the library's error reporting).  Valid until the next call on the same handle/thread. */
const char* qmc_last_error(qmc_system s);

/* Largest delay rank (64, 32, 16, 8 or 4) whose delayed-update chain fits
 * one workgroup's LDS for desc's electron and ion counts and precision (the
 * window of the delayed update of section "Performance and Parallel Scaling"
 * grows as K*N); 1 when none fits
 * (Sherman-Morrison only), 0 for an invalid descriptor.  Host-only: needs no
 * handle; reads the current device's LDS size when a device is present. */
int32_t qmc_max_delay_rank(const qmc_system_desc* desc);

/* Device bytes a handle needs for desc, n_walkers walkers and a gx*gy*gz
 * table (n_orb = max(n_up, n_dn)), including alignment; 0 for invalid input
 * (section "Adapting to trends in High Performance Computing": managing the
 * accelerator's memory explicitly). */
size_t qmc_estimate_device_bytes(const qmc_system_desc* desc, int32_t n_walkers, int32_t gx,
                                 int32_t gy, int32_t gz);

#ifdef __cplusplus
}
#endif

#endif /* QMC_H */
