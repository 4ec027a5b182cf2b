// qmc_kernels.hpp -- host-side launchers of the HIP kernels.  Each returns the
// launch's hipError_t.  Template parameter T: double (FP64) or float (mixed).
#pragma once

#include "qmc_device.hpp"

namespace qmc {

// Ewald-sum constants of one system (splitting parameter kappa, reciprocal
// vectors of one half space with their weights, the ions' structure factor).
constexpr int kEwaldSeg = 10;   // reciprocal vectors per segment of a (Gx, Gy) column

// Real-space Ewald term erfc(kappa r) / r = 1 / r - kappa H(kappa^2 r^2) with the entire
// function H(x) = erf(sqrt x) / sqrt x, tabulated on [0, (kappa rcut)^2] = [0, 5.5^2] as
// degree-kHDeg polynomials in u = (x - x_c) / (kHW / 2) on intervals of width kHW.
// Images other than the minimum one lie at r >= L / 2, i.e. x >= 5.5^2 / 4; there
// erfc(kappa r) / r = kappa G(x) with G(x) = erfc(sqrt x) / sqrt x, tabulated the same way
// on [kGX0, 5.5^2] (no reciprocal square root needed).  G's intervals follow H's.
constexpr int kHDeg = 7;
constexpr double kHW = 0.25;
constexpr int kHInt = 122;                     // covers x < 30.5
constexpr double kGX0 = 7.5;
constexpr int kGInt = 92;                      // covers 7.5 <= x < 30.5
constexpr int kHTab = (kHInt + kGInt) * (kHDeg + 1);    // doubles

struct EwaldParams {
  int enabled;
  int n_g, n_seg;
  double kappa, rcut;
  const double* gvec;    // [n_g][4]: Gx, Gy, Gz, (4 pi / V) exp(-G^2 / 4 kappa^2) / G^2
  const double* s_ion;   // [n_g][2]: sum_I Z_I exp(i G.R_I)
  const int* segs;       // [n_seg][5]: mx, my, mz_lo, mz_hi, index of the first vector in gvec
  const double* htab;    // [kHInt + kGInt][kHDeg + 1]: polynomial coefficients of H, then of G,
                         // lowest degree first
  double c_ee;           // electron self, self-image and background terms
  double c_ei;           // electron-ion background cross term
  double v_ii;           // ion-ion energy (constant)
};

// One system of a batched launch (copied to LDS by each block).
template <typename T>
struct SysDev {
  SysParams P;
  Walkers<T> W;
  EwaldParams E;
  const T* table;
  double* eout;      // [W][4] local energies
  double* mpart;     // [W][np][5] partial sums of the measurement
  int K;             // delay rank of the chain
  int ldl;           // LDS row stride of the inverse
  int tpi_log2;      // gather lanes per proposal (log2)
  int np;            // workgroups per walker in the measurement
  double* scratch;   // [W][bstride] FP64 scratch (rebuild, refinement)
};

// A sweep's proposals in table order (the buffers of one system): the bucket of each item, the
// items sorted by bucket, and the bucket counts and starts.  Buckets are tiles of tile[a] grid
// cells per axis (at most 16 tiles per axis) in Morton order.  hist is zero between sweeps.
constexpr int kGatherBuckets = 4096;
struct GatherOrder {
  int* key;     // [W N]
  int* order;   // [W N]
  int* hist;    // [kGatherBuckets]
  int* offs;    // [kGatherBuckets]
  int tile[3];
};

// Orbital gather: for every (walker, electron), either draw the proposal of
// the sweep in *Wk.sweep_ctr and evaluate all orbitals there (mode 0, written
// to the buffer that does not hold the current row), or evaluate at the
// current position (mode 1, written to buffer 0 and cur reset).
// lanes_log2: lanes per proposal (log2, 0..6); negative = the default for the orbital count.
// sel (nullable): only the walkers w with sel[w] == sel_value are evaluated.
// go (nullable, mode 0): evaluate the proposals in table order (same rows, fewer table misses).
template <typename T>
hipError_t launch_gather(const SysParams& P, const Walkers<T>& Wk, const T* table, int mode, hipStream_t st,
                         int lanes_log2 = -1, const uint32_t* sel = nullptr, uint32_t sel_value = 0,
                         const GatherOrder* go = nullptr);
// Several systems' proposals in one launch; bmap[b] = (system, first item of block b).
template <typename T>
hipError_t launch_gather_batched(const SysDev<T>* sd, const int2* bmap, int n_blocks, hipStream_t st);
int gather_tpi_log2(int nvec);
int gather_items_per_block(int S, size_t tsize);

// Diagnostic evaluation at arbitrary points: out[n][5][n_orb] (FP64).
template <typename T>
hipError_t launch_eval_points(const SysParams& P, const T* table, const double* pos, int n,
                              double* out, hipStream_t st);

// Sequential move chain of one sweep (one workgroup per walker).
template <typename T>
hipError_t launch_chain(const SysParams& P, const Walkers<T>& Wk, hipStream_t st);

// Move chain with rank-K delayed updates (K a power of two, 4..64): per window
// of K moves one product Y = V B0, Schur-complement ratios, one rank-m flush.
// use_mfma selects matrix-core products (else vector ALU).
template <typename T>
hipError_t launch_chain_delayed(const SysParams& P, const Walkers<T>& Wk, int K, int use_mfma, hipStream_t st);
size_t delayed_lds_bytes(const SysParams& P, size_t tsize, bool b_in_lds, int K);
// Whether rank K fits the LDS of one workgroup (single or batched launch) for P.
bool delayed_feasible(const SysParams& P, size_t tsize, int K);
// Batched delayed chain over the systems' walkers; bmap[b] = (system, walker).
// b_in_lds must hold for every system of the launch; lds = dynamic LDS bytes (max).
template <typename T>
hipError_t launch_chain_delayed_batched(const SysDev<T>* sd, const int2* bmap, int n_blocks, bool b_in_lds,
                                        int use_mfma, size_t lds, hipStream_t st);

// Dynamic LDS above 64 KiB needs a per-kernel limit.  allow_dynamic_lds raises it once per
// kernel and device, to what the device allows beside the kernel's static LDS; later calls
// only look it up.  prepare_dynamic_lds raises it for every kernel that can need it, at
// system creation: an attribute call made while another thread captures a graph can
// invalidate that capture, so none is made on the launch path once systems exist.
hipError_t allow_dynamic_lds(const void* kernel);
hipError_t prepare_dynamic_lds();
hipError_t chain_lds_limits();
hipError_t delayed_lds_limits();
hipError_t linalg_lds_limits();
hipError_t measure_lds_limits();
hipError_t drift_lds_limits();

// Particle-by-particle drift-diffusion sweep of every walker (FP64; k_drift.hip): each move's
// orbital row at its proposal is evaluated inside the chain.  sweep: the sweep's index in the
// random streams; crossed (nullable): [W] node-crossing rejections of the sweep (fixed_node).
hipError_t launch_chain_drift(const SysParams& P, const Walkers<double>& Wk, const double* table, uint32_t sweep,
                              int fixed_node, int* crossed, hipStream_t st);
// Whether that chain's LDS (inverse in global memory) fits one workgroup.
bool drift_chain_fits(const SysParams& P);

// Uniform initial positions from the INIT stream of every (walker, electron).
hipError_t launch_init_positions(const SysParams& P, double* pos, hipStream_t st);

// Mixed precision, FP64 fallback of ill-conditioned walkers (k_linalg.hip): mark[w] from the
// measured inverse errors (all != 0: every walker, after a full rebuild); the FP32 rounding
// residual of binv64 for the walkers with mark 1 or 2 (its norm and each column's, with E in
// scratch); the decision, which copies binv = fl32(binv64) for walkers returning to FP32 and
// leaves them mark 3; for those, the measurement's inverse xinv = binv.
hipError_t launch_fb_mark(int W, const double* eta, const int* fb, uint32_t* mark, int all, hipStream_t st);
hipError_t launch_fb_residual(const SysParams& P, const Walkers<float>& Wk, double* scratch, const uint32_t* mark,
                              hipStream_t st);
hipError_t launch_fb_decide(const SysParams& P, const Walkers<float>& Wk, uint32_t* mark, int early, hipStream_t st);
hipError_t launch_fb_adopt(const SysParams& P, const Walkers<float>& Wk, const uint32_t* mark, hipStream_t st);

// Full FP64 inverse of every Slater matrix from the current value rows
// (Gauss-Jordan with partial pivoting); scratch: W * bstride doubles.
// drift (nullable): receives log|D|_old - log|D|_new per [W][2].
// sel (nullable): only walkers w with sel[w] == sel_value are processed, the others keep
// their results.  beside: the launch runs beside another kernel that fills the device (a
// selective rebuild then takes the 256-thread panel elimination, which is placed beside the
// other kernel's workgroups; alone, the register elimination is faster).  Mixed precision:
// the FP64 inverse goes to binv64 as well.
template <typename T>
hipError_t launch_rebuild(const SysParams& P, const Walkers<T>& Wk, double* scratch, double* drift,
                          hipStream_t st, const uint32_t* sel = nullptr, uint32_t sel_value = 0,
                          bool beside = false);

// Mixed precision: Wk.xinv = B + B (I - A B) with the FP64 Slater matrix A (from val64) and
// FP64 products, the inverse the measurement reads; eta = ||I - A B||_F and ||X||_F per spin;
// scratch: W * bstride doubles.  FP64 fallback walkers are skipped; sel (nullable): only the
// walkers with sel[w] == sel_value.
template <typename T>
hipError_t launch_refine(const SysParams& P, const Walkers<T>& Wk, double* scratch, hipStream_t st,
                         const uint32_t* sel = nullptr, uint32_t sel_value = 0);
// Batched refinement of every (system, walker) of fmap, both spins.
template <typename T>
hipError_t launch_refine_batched(const SysDev<T>* sd, const int2* fmap, int n_walkers, hipStream_t st);

// Local energy of every walker: out[W][4]; partial: W * kMaxMeasureParts * 5 doubles of scratch.
constexpr int kMaxMeasureParts = 8;
template <typename T>
hipError_t launch_measure(const SysParams& P, const Walkers<T>& Wk, const EwaldParams& E, double* partial,
                          double* out, hipStream_t st);
// Workgroups per walker the measurement uses for W walkers (a power of two, at most kMaxMeasureParts).
int measure_parts(int W);
// Batched measurement: bmap[b] = (system, walker * np + part) per workgroup, then fmap[t] =
// (system, walker) for the n_walkers sums; lds = dynamic LDS bytes (max over systems).
template <typename T>
hipError_t launch_measure_batched(const SysDev<T>* sd, const int2* bmap, int n_blocks, const int2* fmap,
                                  int n_walkers, size_t lds, hipStream_t st);
size_t measure_lds_bytes(const SysParams& P, int np);

// All-electron moves: the state at the proposed configuration R' of every walker.
template <typename T>
struct AeProposal {
  T* binv;          // [W][bstride]: inverses at R' (written by the rebuild with row_flip = 1)
  double* logdet;   // [W][2]: log|D(R')| per spin (NaN when singular)
  int* sign;        // [W][2]
  int* status;      // [W]: nonzero = a singular matrix at R'
  double* dj;       // [W][dj_parts]: partial sums of J(R') - J(R)
  double* logT;     // [W][logT_parts] or null: partial sums of log T(R' -> R) / T(R -> R') of
                    // drift-diffusion proposals, added in order by the decision
  int logT_parts;
  int dj_parts;
  int fixed_node;   // 1: reject moves that change the sign of Psi (diffusion Monte Carlo)
  int* crossed;     // [W] or null: 1 where the move was rejected for crossing a node
  const double* vprop;  // [W][N][3] or null: drift velocities at R', which become those at R
  double* vcur;         //   (vcur) of an accepted walker
  double* binv64;       // [W][bstride] or null: FP64 inverses at R' (mixed precision, drift
                        //   moves), which become the current ones of an accepted walker
};
// dj[w][jastrow_parts(N)] = partial sums of J(R') - J(R) from pos and the proposals; clears
// status_prop.
int jastrow_parts(int N);
hipError_t launch_ae_jastrow(const SysParams& P, const double* pos, const double* prop, double* dj,
                             int* status_prop, hipStream_t st);
// Drift velocities grad ln|Psi| of every electron at R (prop = 0) or R' (prop = 1, also
// A.logT from vcur = v(R), A.logT_parts == velocity_parts(N)); vel, vcur: [W][N][3].  N at
// most 1024.
int velocity_parts(int N);
template <typename T>
hipError_t launch_ae_velocity(const SysParams& P, const Walkers<T>& Wk, const AeProposal<T>& A, int prop,
                              double* vel, const double* vcur, hipStream_t st);
// Accept or reject every walker's all-electron move and install R' on acceptance.
template <typename T>
hipError_t launch_ae_apply(const SysParams& P, const Walkers<T>& Wk, const AeProposal<T>& A, hipStream_t st);

// Diffusion Monte Carlo population of W slots (a slot is alive while its weight is > 0).
struct DmcState {
  double* w;        // [W] weights
  double* E;        // [W] local energy of each slot's current configuration
  double* wb;       // [W][2] the step's weight and local energy before branching (0 and NaN
                    // for slots that were dead when the step began)
  const double* e4; // [W][4] the step's local energies (kinetic, e-e, e-I, I-I)
  const int* crossed;  // [W] node-crossing rejections of the step
  int* mult;        // [W] branching multiplicities
  int* plan;        // [W] source slot of the copy placed in each slot, or -1
  int* xscan;       // [W] exclusive prefix sums of the extra copies
  int* fscan;       // [W] exclusive prefix sums of the free slots
  double* ctl;      // [2]: E_T, feedback
  int* ictl;        // [3]: step, extinct flag, target population
  double* stats;    // [6] of this step: E, sum w, population, E_T used, dropped copies, crossings
  double* vel;      // [W][N][3] or null: drift velocities at each slot's configuration (copied along)
};
// Weights, estimator, multiplicities, copy plan, new weights and E_T of one DMC step (one
// workgroup), then the walker states of the copies.
hipError_t launch_dmc_branch(const SysParams& P, const DmcState& D, hipStream_t st);
template <typename T>
hipError_t launch_dmc_copy(const SysParams& P, const Walkers<T>& Wk, const DmcState& D, hipStream_t st);

// Size in bytes of the dynamic LDS the chain kernel needs for P.
size_t chain_lds_bytes(const SysParams& P, size_t tsize, bool b_in_lds);

}  // namespace qmc
