// capi.hip -- the C ABI (include/qmc.h): handle lifetime, device memory,
// set-up tables and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "qmc_kernels.hpp"

using namespace qmc;

namespace {

thread_local std::string g_last_error;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Device memory of a handle: either hipMalloc'd buffers or a bump region of
// the caller's arena.  mark()/release_to() let the walker region be rebuilt.
struct DeviceMemory {
  char* arena = nullptr;
  size_t arena_bytes = 0, used = 0;
  struct Block { void* p; size_t mark; };
  std::vector<Block> blocks;
  hipError_t last = hipSuccess;

  void* alloc(size_t bytes) {
    bytes = align_up(bytes ? bytes : 1);
    if (arena) {
      if (used + bytes > arena_bytes) return nullptr;
      void* p = arena + used;
      blocks.push_back({p, used});
      used += bytes;
      return p;
    }
    void* p = nullptr;
    last = hipMalloc(&p, bytes);
    if (last != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    blocks.push_back({p, used});
    used += bytes;
    return p;
  }
  size_t mark() const { return blocks.size(); }
  void release_to(size_t m) {
    while (blocks.size() > m) {
      Block b = blocks.back();
      blocks.pop_back();
      if (!arena) (void)hipFree(b.p);
      used = b.mark;
    }
  }
};

struct TimerClass {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> live, pool;
  double ms = 0.0;
  int64_t launches = 0;
};

size_t tsize_of(int precision) { return precision == QMC_MIXED ? sizeof(float) : sizeof(double); }

int padded_stride(int n_orb, int precision) {
  const int v = precision == QMC_MIXED ? 4 : 2;   // 16-byte vectors
  return (n_orb + v - 1) / v * v;
}

}  // namespace

struct qmc_system_s {
  qmc_system_desc d{};
  std::vector<double> ions4;             // [n_ions][4]
  std::vector<double> j2p, j1p;
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  DeviceMemory mem;
  size_t mark_sys = 0, mark_table = 0;
  SysParams P{};
  EwaldParams E{};
  double* d_ions = nullptr;
  double* d_gvec = nullptr;
  double* d_sion = nullptr;
  int* d_segs = nullptr;
  double* d_htab = nullptr;
  void* d_table = nullptr;
  bool has_table = false, has_walkers = false;
  uint32_t sweep_index = 0;
  // walker buffers (untyped; T per precision)
  double* pos = nullptr;
  double* prop = nullptr;
  void* vgl = nullptr;
  uint8_t* cur = nullptr;
  void* binv = nullptr;
  double* logdet = nullptr;
  int* sign = nullptr;
  uint8_t* acc = nullptr;
  uint32_t* nacc = nullptr;
  int* status = nullptr;
  double* val64 = nullptr;
  void* xinv = nullptr;      // FP64-refined inverse read by the measurement (mixed precision)
  // mixed precision: FP64 inverses (particle-by-particle moves: of the FP64 fallback walkers;
  // drift moves: of every walker, with the FP64 gradient rows, for the velocities)
  double* binv64 = nullptr;
  double* grad64 = nullptr;
  double* ae_binv64 = nullptr;   // drift moves: FP64 inverses at R'
  // mixed precision, particle-by-particle moves: FP64 fallback of ill-conditioned walkers
  int* fb = nullptr;
  double* eta = nullptr;
  float* ecol = nullptr;
  uint32_t* eta_age = nullptr;
  uint32_t* pstat = nullptr;
  uint32_t* fbmark = nullptr;
  int gather_lanes_log2 = -1;   // lanes per proposal in the gather (log2); -1 = default
  // the sweep's proposals evaluated in table order (null: in (walker, electron) order)
  GatherOrder gorder{};
  bool gather_ordered = false;
  uint32_t* nguard = nullptr;
  uint32_t* sweep_ctr = nullptr;
  // all-electron moves: the state at the proposed configurations (null for particle-by-particle)
  void* ae_binv = nullptr;
  double* ae_logdet = nullptr;
  double* ae_dj = nullptr;
  int* ae_sign = nullptr;
  int* ae_status = nullptr;
  double* ae_vcur = nullptr;   // drift moves: velocities at R, at R', and the transition-ratio logs
  double* ae_vprop = nullptr;
  double* ae_logT = nullptr;
  // diffusion Monte Carlo population (allocated by qmc_dmc_init)
  bool dmc_ready = false, fixed_node = false;
  bool vcur_valid = false;   // drift moves: ae_vcur holds the velocities at the current configuration
  double* dmc_w = nullptr;
  double* dmc_E = nullptr;
  double* dmc_e4 = nullptr;
  double* dmc_wb = nullptr;   // [W][2] weight and energy before the last branching
  double* dmc_ctl = nullptr;
  int* dmc_i = nullptr;   // crossed, mult, plan, xscan, fscan ([W] each), then the 3 control ints
  double* scratch = nullptr;
  double* drift = nullptr;
  double* energy = nullptr;
  bool timing = false;
  int use_mfma = 1;   // delayed-update products on the matrix cores (QMC_DELAYED_VALU=1: vector ALU)
  TimerClass timers[4];
  hipStream_t side = nullptr;              // measurements of qmc_run_steps (created on first use)
  hipEvent_t ev_swept = nullptr, ev_measured = nullptr;
};

namespace {

qmc_status fail(qmc_system s, qmc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  if (s) s->err = buf;
  return st;
}

#define HIP_TRY(s, expr)                                                                     \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((s), QMC_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

template <typename T>
Walkers<T> walkers_of(qmc_system s) {
  Walkers<T> w;
  w.pos = s->pos; w.prop = s->prop; w.vgl = static_cast<T*>(s->vgl); w.cur = s->cur;
  w.binv = static_cast<T*>(s->binv); w.logdet = s->logdet; w.sign = s->sign; w.acc = s->acc;
  w.nacc = s->nacc; w.status = s->status; w.val64 = s->val64; w.nguard = s->nguard; w.sweep_ctr = s->sweep_ctr;
  w.xinv = static_cast<T*>(s->xinv);
  w.row_flip = 0;
  w.drift_v = s->d.move_kind == QMC_MOVE_ALL_DRIFT ? s->ae_vcur : nullptr;
  w.vstride = kComp * s->P.S;
  w.binv64 = s->binv64;
  w.fb = s->fb;
  w.fb_sel = 0;
  w.eta = s->eta;
  w.ecol = s->ecol;
  w.eta_age = s->eta_age;
  w.pstat = s->pstat;
  w.table = static_cast<const T*>(s->d_table);
  w.grad64 = s->grad64;
  return w;
}

// The FP64 view of a mixed system's fallback walkers: the chain runs on the FP64 value rows
// and the FP64 inverses of the walkers with fb[w] = 1.
Walkers<double> fallback_of(qmc_system s) {
  Walkers<double> w = walkers_of<double>(s);
  w.vgl = s->val64;
  w.vstride = s->P.S;
  w.binv = s->binv64;
  w.val64 = nullptr;
  w.xinv = nullptr;
  w.binv64 = nullptr;
  w.fb_sel = 1;
  w.eta = nullptr;
  w.ecol = nullptr;
  w.eta_age = nullptr;
  w.table = nullptr;
  return w;
}

bool uses_fallback(qmc_system s) { return s->d.precision == QMC_MIXED && s->d.move_kind == QMC_MOVE_PBYP; }

// Event-bracketed launch: f() issues the kernel on s->stream.
template <typename F>
hipError_t timed(qmc_system s, int cls, F&& f, hipStream_t st);

// Event-bracketed launch on the handle's stream.
template <typename F>
hipError_t timed(qmc_system s, int cls, F&& f) {
  return timed(s, cls, static_cast<F&&>(f), s->stream);
}

template <typename F>
hipError_t timed(qmc_system s, int cls, F&& f, hipStream_t st) {
  if (!s->timing) return f();
  TimerClass& tc = s->timers[cls];
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (!tc.pool.empty()) { ev = tc.pool.back(); tc.pool.pop_back(); }
  else {
    hipError_t e = hipEventCreate(&ev.first);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&ev.second);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipEventRecord(ev.first, st);
  if (e != hipSuccess) return e;
  e = f();
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev.second, st);
  tc.live.push_back(ev);
  return e;
}

void build_radial(Radial& R, int kind, const double* p, int M, double rc, double cusp, double a, double b) {
  std::memset(&R, 0, sizeof R);
  R.kind = kind;
  if (kind == QMC_J_PADE) { R.a = a; R.b = b; }
  if (kind == QMC_J_BSPLINE) {
    R.M = M;
    R.rc = rc;
    R.inv_delta = M / rc;
    for (int m = 1; m <= M; ++m) R.p[m] = p[m - 1];
    R.p[0] = R.p[2] - 2.0 * (rc / M) * cusp;   // u'(0) = (p_2 - p_0) / (2 rc / M)
  }
}

// Ewald tables (section "Long-Range Interactions").  Splitting kappa = 5.5 / L
// with the real-space cutoff at one cell side L (erfc(5.5) ~ 7e-15), and every
// reciprocal vector of one half space with G^2 / (4 kappa^2) <= 30, grouped in
// segments of at most kEwaldSeg consecutive Gz of one (Gx, Gy) column.
// H(x) = erf(sqrt x) / sqrt x (its series near 0), for the real-space table.
double erf_over_sqrt(double x) {
  if (x < 1e-10) return 2.0 / std::sqrt(kPi) * (1.0 - x / 3.0);
  const double r = std::sqrt(x);
  return std::erf(r) / r;
}

// G(x) = erfc(sqrt x) / sqrt x, for images beyond the minimum one (x >= kGX0 > 0).
double erfc_over_sqrt(double x) {
  const double r = std::sqrt(x);
  return std::erfc(r) / r;
}

// Coefficients of f on n_int intervals of width kHW from x0: Chebyshev interpolation at
// kHDeg + 1 Chebyshev points of each interval, rewritten in powers of the interval's
// scaled variable u.
void fit_intervals(double (*f)(double), double x0, int n_int, double* tab) {
  constexpr int D = kHDeg, M = kHDeg + 1;
  double T[M][M] = {};   // T[j][m]: coefficient of u^m in the Chebyshev polynomial T_j
  T[0][0] = 1.0;
  if (D >= 1) T[1][1] = 1.0;
  for (int j = 2; j <= D; ++j)
    for (int m = 0; m <= D; ++m) T[j][m] = (m > 0 ? 2.0 * T[j - 1][m - 1] : 0.0) - T[j - 2][m];
  for (int i = 0; i < n_int; ++i) {
    const double xc = x0 + (i + 0.5) * kHW;
    double fv[M], a[M];
    for (int k = 0; k < M; ++k) fv[k] = f(xc + 0.5 * kHW * std::cos(kPi * (k + 0.5) / M));
    for (int j = 0; j < M; ++j) {
      double acc = 0.0;
      for (int k = 0; k < M; ++k) acc += fv[k] * std::cos(j * kPi * (k + 0.5) / M);
      a[j] = (j == 0 ? 1.0 : 2.0) * acc / M;
    }
    for (int m = 0; m <= D; ++m) tab[(size_t)i * M + m] = 0.0;
    for (int j = 0; j < M; ++j)
      for (int m = 0; m <= D; ++m) tab[(size_t)i * M + m] += a[j] * T[j][m];
  }
}

void h_table(std::vector<double>& tab) {
  tab.assign(kHTab, 0.0);
  fit_intervals(erf_over_sqrt, 0.0, kHInt, tab.data());
  fit_intervals(erfc_over_sqrt, kGX0, kGInt, tab.data() + (size_t)kHInt * (kHDeg + 1));
}

void ewald_setup(qmc_system s, std::vector<double>& gvec, std::vector<double>& sion,
                 std::vector<int>& segs) {
  const double L = s->d.L, V = L * L * L;
  const double kappa = 5.5 / L;
  const double g0 = 2.0 * kPi / L;
  const double gmax2 = 30.0 * 4.0 * kappa * kappa;
  const int m2max = (int)std::floor(gmax2 / (g0 * g0));
  const int mmax = (int)std::floor(std::sqrt((double)m2max));
  const int M = s->d.n_ions;
  for (int a = 0; a <= mmax; ++a)
    for (int b = -mmax; b <= mmax; ++b) {
      if (a == 0 && b < 0) continue;                 // one of each +-G pair
      const int rem = m2max - a * a - b * b;
      if (rem < 0) continue;
      const int cm = (int)std::floor(std::sqrt((double)rem));
      const int lo = (a == 0 && b == 0) ? 1 : -cm;
      for (int c0 = lo; c0 <= cm; c0 += kEwaldSeg) {
        const int c1 = std::min(cm, c0 + kEwaldSeg - 1);
        segs.push_back(a); segs.push_back(b); segs.push_back(c0); segs.push_back(c1);
        segs.push_back((int)(gvec.size() / 4));
        for (int c = c0; c <= c1; ++c) {
          const double Gx = g0 * a, Gy = g0 * b, Gz = g0 * c;
          const double G2 = Gx * Gx + Gy * Gy + Gz * Gz;
          gvec.push_back(Gx); gvec.push_back(Gy); gvec.push_back(Gz);
          gvec.push_back(4.0 * kPi / V * std::exp(-G2 / (4.0 * kappa * kappa)) / G2);
          double re = 0.0, im = 0.0;
          for (int I = 0; I < M; ++I) {
            const double ph = Gx * s->ions4[4 * I] + Gy * s->ions4[4 * I + 1] + Gz * s->ions4[4 * I + 2];
            re += s->ions4[4 * I + 3] * std::cos(ph);
            im += s->ions4[4 * I + 3] * std::sin(ph);
          }
          sion.push_back(re); sion.push_back(im);
        }
      }
    }
  // self-image sum: sum_{n != 0} erfc(kappa |n| L) / (|n| L)
  double simg = 0.0;
  for (int a = -2; a <= 2; ++a)
    for (int b = -2; b <= 2; ++b)
      for (int c = -2; c <= 2; ++c) {
        if (!a && !b && !c) continue;
        const double r = L * std::sqrt((double)(a * a + b * b + c * c));
        simg += std::erfc(kappa * r) / r;
      }
  const double N = s->d.n_up + s->d.n_dn;
  double Zt = 0.0, Z2 = 0.0;
  for (int I = 0; I < M; ++I) { Zt += s->ions4[4 * I + 3]; Z2 += s->ions4[4 * I + 3] * s->ions4[4 * I + 3]; }
  s->E.kappa = kappa;
  s->E.rcut = L;
  s->E.n_g = (int)(gvec.size() / 4);
  s->E.n_seg = (int)(segs.size() / 5);
  s->E.c_ee = -kappa / std::sqrt(kPi) * N + 0.5 * N * simg - kPi * N * N / (2.0 * V * kappa * kappa);
  s->E.c_ei = kPi * N * Zt / (V * kappa * kappa);
  // ions alone: pairs over every image closer than the cutoff, reciprocal, self and background
  double vii = 0.0;
  for (int I = 0; I < M; ++I)
    for (int J = 0; J < M; ++J) {
      if (I == J) continue;
      double d[3];
      for (int k = 0; k < 3; ++k) {
        const double x = s->ions4[4 * I + k] - s->ions4[4 * J + k];
        d[k] = x - L * std::rint(x / L);
      }
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
          for (int c = -1; c <= 1; ++c) {
            const double x = d[0] + a * L, y = d[1] + b * L, z = d[2] + c * L;
            const double r = std::sqrt(x * x + y * y + z * z);
            if (r < s->E.rcut) vii += 0.5 * s->ions4[4 * I + 3] * s->ions4[4 * J + 3] * std::erfc(kappa * r) / r;
          }
    }
  for (size_t g = 0; g < sion.size() / 2; ++g)
    vii += gvec[4 * g + 3] * (sion[2 * g] * sion[2 * g] + sion[2 * g + 1] * sion[2 * g + 1]);
  vii += -kappa / std::sqrt(kPi) * Z2 + 0.5 * Z2 * simg - kPi * Zt * Zt / (2.0 * V * kappa * kappa);
  s->E.v_ii = M ? vii : 0.0;
}

void free_walkers(qmc_system s) {
  s->mem.release_to(s->mark_table);
  s->has_walkers = false;
  s->pos = s->prop = nullptr;
  s->gorder = GatherOrder{};
  s->gather_ordered = false;
  s->vgl = s->binv = nullptr;
  s->cur = s->acc = nullptr;
  s->logdet = s->scratch = s->drift = s->energy = nullptr;
  s->sign = s->status = nullptr;
  s->nacc = nullptr;
  s->val64 = nullptr;
  s->xinv = nullptr;
  s->binv64 = s->eta = s->grad64 = s->ae_binv64 = nullptr;
  s->ecol = nullptr;
  s->fb = nullptr;
  s->eta_age = s->pstat = s->fbmark = nullptr;
  s->nguard = nullptr;
  s->sweep_ctr = nullptr;
  s->ae_binv = nullptr;
  s->ae_logdet = s->ae_dj = nullptr;
  s->ae_sign = s->ae_status = nullptr;
  s->ae_vcur = s->ae_vprop = s->ae_logT = nullptr;
  s->dmc_ready = s->fixed_node = false;
  s->vcur_valid = false;
  s->dmc_w = s->dmc_E = s->dmc_e4 = s->dmc_wb = s->dmc_ctl = nullptr;
  s->dmc_i = nullptr;
}

struct WalkerSizes {
  size_t pos, prop, vgl, cur, binv, logdet, sign, acc, nacc, status, scratch, drift, energy, val64, nguard, sweep,
      xinv, binv64, fb, eta, ecol, eta_age, pstat, fbmark, ae_binv, ae_logdet, ae_dj, ae_sign, ae_status, ae_vel, ae_logT,
      grad64, ae_binv64, dmc, gitem, gbucket;
  size_t total() const {
    return 2 * align_up(gitem) + 2 * align_up(gbucket) +
           align_up(pos) + align_up(prop) + align_up(vgl) + align_up(cur) + align_up(binv) +
           align_up(logdet) + align_up(sign) + align_up(acc) + align_up(nacc) + align_up(status) +
           align_up(scratch) + align_up(drift) + align_up(energy) + align_up(val64) + align_up(nguard) +
           align_up(sweep) + align_up(xinv) +
           align_up(binv64) + align_up(grad64) + align_up(ae_binv64) +
           (fb ? align_up(fb) + align_up(eta) + align_up(ecol) + align_up(eta_age) + align_up(pstat) +
                     align_up(fbmark)
               : 0) +
           (ae_binv ? align_up(ae_binv) + align_up(ae_logdet) + align_up(ae_dj) + align_up(ae_sign) +
                          align_up(ae_status)
                    : 0) +
           (ae_vel ? 2 * align_up(ae_vel) + align_up(ae_logT) : 0) + dmc;
  }
};

WalkerSizes walker_sizes(int n_up, int n_dn, int precision, int W, int n_orb, int move_kind) {
  const size_t N = (size_t)n_up + n_dn, S = padded_stride(n_orb, precision), ts = tsize_of(precision);
  const size_t bs = (size_t)n_up * n_up + (size_t)n_dn * n_dn;
  WalkerSizes z;
  z.pos = W * N * 3 * sizeof(double);
  z.prop = W * N * 4 * sizeof(double);
  // the gather's table order (every move kind whose proposals a gather evaluates)
  const bool gathers = move_kind != QMC_MOVE_PBYP_DRIFT && W * N < ((size_t)1 << 31);
  z.gitem = gathers ? W * N * sizeof(int) : 0;
  z.gbucket = gathers ? kGatherBuckets * sizeof(int) : 0;
  z.vgl = 2 * W * N * kComp * S * ts;
  z.cur = W * N;
  z.binv = W * bs * ts;
  z.logdet = W * 2 * sizeof(double);
  z.sign = W * 2 * sizeof(int);
  z.acc = W * N;
  z.nacc = W * sizeof(uint32_t);
  z.status = W * sizeof(int);
  z.scratch = W * bs * sizeof(double);
  z.drift = W * 2 * sizeof(double);
  z.energy = W * (4 + kMaxMeasureParts * 5) * sizeof(double);   // energies, then measurement partials
  z.val64 = precision == QMC_MIXED ? 2 * W * N * S * sizeof(double) : 0;
  z.xinv = precision == QMC_MIXED ? W * bs * ts : 0;
  const bool fbk = precision == QMC_MIXED && move_kind == QMC_MOVE_PBYP;   // FP64 fallback state
  // mixed precision with drift moves: FP64 gradient rows and FP64 inverses at R and R', so the
  // drift velocities (the proposals' centres and the transition ratios) are FP64 quantities
  const bool mdrift = precision == QMC_MIXED && move_kind == QMC_MOVE_ALL_DRIFT;
  z.binv64 = fbk || mdrift ? W * bs * sizeof(double) : 0;
  z.grad64 = mdrift ? 2 * W * N * 3 * S * sizeof(double) : 0;
  z.ae_binv64 = mdrift ? W * bs * sizeof(double) : 0;
  z.fb = fbk ? W * sizeof(int) : 0;
  z.eta = fbk ? W * 4 * sizeof(double) : 0;
  z.ecol = fbk ? W * N * sizeof(float) : 0;
  z.eta_age = fbk ? W * sizeof(uint32_t) : 0;
  z.pstat = fbk ? W * 2 * sizeof(uint32_t) : 0;
  z.fbmark = fbk ? W * sizeof(uint32_t) : 0;
  z.nguard = W * sizeof(uint32_t);
  z.sweep = sizeof(uint32_t);
  const bool ae = move_kind == QMC_MOVE_ALL || move_kind == QMC_MOVE_ALL_DRIFT;
  z.ae_binv = ae ? W * bs * ts : 0;
  z.ae_logdet = ae ? W * 2 * sizeof(double) : 0;
  z.ae_dj = ae ? W * (size_t)jastrow_parts((int)N) * sizeof(double) : 0;
  z.ae_sign = ae ? W * 2 * sizeof(int) : 0;
  z.ae_status = ae ? W * sizeof(int) : 0;
  const bool drift = move_kind == QMC_MOVE_ALL_DRIFT;
  const bool dmc_ok = drift || move_kind == QMC_MOVE_PBYP_DRIFT;   // moves DMC can run on
  z.ae_vel = drift ? W * N * 3 * sizeof(double) : 0;
  z.ae_logT = drift ? W * (size_t)velocity_parts((int)N) * sizeof(double) : 0;
  // the DMC population qmc_dmc_init carves out (weights, energies, [W][4] energies, [W][2]
  // weights and energies before branching, control doubles, five [W] int arrays and the
  // control ints)
  z.dmc = dmc_ok ? align_up(W * sizeof(double)) * 2 + align_up(W * 4 * sizeof(double)) +
                      align_up(W * 2 * sizeof(double)) + align_up(2 * sizeof(double)) +
                      align_up((5 * (size_t)W + 3) * sizeof(int))
                : 0;
  return z;
}

size_t system_bytes(const qmc_system_desc* d) {
  // ions + Ewald tables (upper bounds on the reciprocal list and its segments)
  const int mmax = (int)std::ceil(std::sqrt(120.0) * 5.5 / (2.0 * kPi));
  const size_t ng = (size_t)(mmax + 1) * (2 * mmax + 1) * (2 * mmax + 1);
  const size_t nseg = (size_t)(mmax + 1) * (2 * mmax + 1) * 3;
  return align_up((size_t)(d->n_ions > 0 ? d->n_ions : 1) * 4 * sizeof(double)) +
         align_up(ng * 4 * sizeof(double)) + align_up(ng * 2 * sizeof(double)) +
         align_up(nseg * 5 * sizeof(int)) + align_up(kHTab * sizeof(double));
}

bool valid_rank(int K) { return K == 0 || K == 1 || (K >= 4 && K <= 64 && !(K & (K - 1))); }

qmc_status validate(const qmc_system_desc* d) {
  if (!d) return fail(nullptr, QMC_ERR_ARG, "desc is NULL");
  if (d->n_up < 1 || d->n_dn < 0 || d->n_up + d->n_dn > 1024)
    return fail(nullptr, QMC_ERR_ARG, "need n_up >= 1, n_dn >= 0, n_up + n_dn <= 1024");
  if (!(d->L > 0.0) || !std::isfinite(d->L)) return fail(nullptr, QMC_ERR_ARG, "L must be positive");
  if (!(d->sigma > 0.0)) return fail(nullptr, QMC_ERR_ARG, "sigma must be positive");
  if (d->precision != QMC_FP64 && d->precision != QMC_MIXED)
    return fail(nullptr, QMC_ERR_ARG, "unknown precision %d", d->precision);
  if (!valid_rank(d->delay_rank))
    return fail(nullptr, QMC_ERR_ARG, "delay_rank %d: use 1 (Sherman-Morrison) or a power of two in [4, 64]",
                d->delay_rank);
  if (d->recompute_period < 0) return fail(nullptr, QMC_ERR_ARG, "recompute_period must be >= 0");
  if (d->move_kind != QMC_MOVE_PBYP && d->move_kind != QMC_MOVE_ALL && d->move_kind != QMC_MOVE_ALL_DRIFT &&
      d->move_kind != QMC_MOVE_PBYP_DRIFT)
    return fail(nullptr, QMC_ERR_ARG, "unknown move_kind %d", d->move_kind);
  if (d->move_kind == QMC_MOVE_PBYP_DRIFT && d->precision != QMC_FP64)
    return fail(nullptr, QMC_ERR_ARG, "particle-by-particle drift moves run in FP64 (precision QMC_FP64)");
  if (d->hamiltonian != QMC_H_KINETIC && d->hamiltonian != QMC_H_COULOMB_EWALD)
    return fail(nullptr, QMC_ERR_ARG, "unknown hamiltonian %d", d->hamiltonian);
  if (d->n_ions < 0 || (d->n_ions > 0 && (!d->ion_pos || !d->ion_Z)))
    return fail(nullptr, QMC_ERR_ARG, "n_ions > 0 needs ion_pos and ion_Z");
  if (d->n_ions > 4096) return fail(nullptr, QMC_ERR_ARG, "at most 4096 ions");
  auto check_j = [&](int kind, const double* p, int n, double rc, const char* nm) -> qmc_status {
    if (kind == QMC_J_NONE) return QMC_OK;
    if (kind == QMC_J_PADE) {
      if (!p || n != 2) return fail(nullptr, QMC_ERR_ARG, "%s Pade needs params {a, b}", nm);
      return QMC_OK;
    }
    if (kind == QMC_J_BSPLINE) {
      if (!p || n < 2 || n > QMC_MAX_KNOTS)
        return fail(nullptr, QMC_ERR_ARG, "%s B-spline needs 2..%d control points", nm, QMC_MAX_KNOTS);
      if (!(rc > 0.0) || rc > 0.5 * d->L * (1.0 + 1e-12))
        return fail(nullptr, QMC_ERR_ARG, "%s cutoff must be in (0, L/2]", nm);
      return QMC_OK;
    }
    return fail(nullptr, QMC_ERR_ARG, "%s: unknown kind %d", nm, kind);
  };
  qmc_status st = check_j(d->j2_kind, d->j2_params, d->j2_n, d->j2_rcut, "j2");
  if (st != QMC_OK) return st;
  if (d->j1_kind == QMC_J_PADE) return fail(nullptr, QMC_ERR_ARG, "j1 supports NONE or BSPLINE");
  st = check_j(d->j1_kind, d->j1_params, d->j1_n, d->j1_rcut, "j1");
  if (st != QMC_OK) return st;
  if (d->j3_gamma) {
    const int L3 = d->j3_m_ei, M3 = d->j3_m_ee;
    if (d->n_ions < 1) return fail(nullptr, QMC_ERR_ARG, "the three-body term needs ions");
    if (L3 < 0 || L3 > 3 || M3 < 0 || M3 > 3) return fail(nullptr, QMC_ERR_ARG, "three-body orders must be in [0, 3]");
    if (!(d->j3_rcut > 0.0) || d->j3_rcut > 0.5 * d->L * (1.0 + 1e-12))
      return fail(nullptr, QMC_ERR_ARG, "three-body cutoff must be in (0, L/2]");
    for (int sp = 0; sp < 2; ++sp)
      for (int l = 0; l <= L3; ++l)
        for (int m = 0; m <= L3; ++m)
          for (int n = 0; n <= M3; ++n) {
            const double* g = d->j3_gamma + (size_t)sp * (L3 + 1) * (L3 + 1) * (M3 + 1);
            const double x = g[((size_t)l * (L3 + 1) + m) * (M3 + 1) + n];
            if (!std::isfinite(x) || x != g[((size_t)m * (L3 + 1) + l) * (M3 + 1) + n])
              return fail(nullptr, QMC_ERR_ARG, "three-body coefficients must be finite with g_lmn = g_mln");
          }
  }
  return QMC_OK;
}

}  // namespace

namespace qmc {

hipError_t allow_dynamic_lds(const void* kernel) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({kernel, dev})) return hipSuccess;
  hipFuncAttributes a;
  e = hipFuncGetAttributes(&a, kernel);
  if (e != hipSuccess) return e;
  int max = 0;
  e = hipDeviceGetAttribute(&max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, max - (int)a.sharedSizeBytes);
  if (e == hipSuccess) done.insert({kernel, dev});
  return e;
}

hipError_t prepare_dynamic_lds() {
  hipError_t e = chain_lds_limits();
  if (e == hipSuccess) e = delayed_lds_limits();
  if (e == hipSuccess) e = linalg_lds_limits();
  if (e == hipSuccess) e = measure_lds_limits();
  if (e == hipSuccess) e = drift_lds_limits();
  return e;
}

}  // namespace qmc

extern "C" {


qmc_status qmc_create_system(const qmc_system_desc* desc, void* hip_stream, qmc_system* out) {
  if (!out) return fail(nullptr, QMC_ERR_ARG, "out is NULL");
  *out = nullptr;
  qmc_status st = validate(desc);
  if (st != QMC_OK) return st;
  qmc_system s = new (std::nothrow) qmc_system_s;
  if (!s) return fail(nullptr, QMC_ERR_OOM, "host allocation failed");
  s->d = *desc;
  s->d.j3_gamma = nullptr;   // copied to the device below; the caller's array is not kept
  if (s->d.delay_rank == 0) s->d.delay_rank = 1;
  {
    const char* v = getenv("QMC_DELAYED_VALU");
    s->use_mfma = !(v && v[0] == '1');
  }
  s->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(nullptr, QMC_ERR_DEVICE, "no HIP device");
  }
  {
    const hipError_t e = prepare_dynamic_lds();
    if (e != hipSuccess) {
      delete s;
      return fail(nullptr, QMC_ERR_DEVICE, "raising the kernels' dynamic LDS limits failed: %s", hipGetErrorString(e));
    }
  }
  if (desc->arena) {
    s->mem.arena = static_cast<char*>(desc->arena);
    s->mem.arena_bytes = desc->arena_bytes;
  }
  const int M = desc->n_ions;
  s->ions4.resize((size_t)(M > 0 ? M : 1) * 4, 0.0);
  for (int I = 0; I < M; ++I) {
    for (int k = 0; k < 3; ++k) {
      const double x = desc->ion_pos[3 * I + k];
      double y = x - desc->L * std::floor(x / desc->L);
      if (y >= desc->L) y = 0.0;
      s->ions4[4 * I + k] = y;
    }
    s->ions4[4 * I + 3] = desc->ion_Z[I];
  }
  // parameters copied into the handle
  SysParams& P = s->P;
  std::memset(&P, 0, sizeof P);
  P.n_up = desc->n_up;
  P.n_dn = desc->n_dn;
  P.N = desc->n_up + desc->n_dn;
  P.n_orb = desc->n_up > desc->n_dn ? desc->n_up : desc->n_dn;
  P.S = padded_stride(P.n_orb, desc->precision);
  P.n_ions = M;
  P.bstride = desc->n_up * desc->n_up + desc->n_dn * desc->n_dn;
  P.L = desc->L;
  P.sigma = desc->sigma;
  P.tie_guard = desc->tie_guard > 0.0 ? desc->tie_guard : 1e-3;
  P.key0 = (uint32_t)desc->seed;
  P.key1 = (uint32_t)(desc->seed >> 32);
  const double* j2p = desc->j2_params;
  build_radial(P.jas.same, desc->j2_kind, j2p, desc->j2_n, desc->j2_rcut, desc->j2_cusp_same,
               j2p ? j2p[0] : 0.0, (j2p && desc->j2_n > 1) ? j2p[1] : 0.0);
  build_radial(P.jas.opp, desc->j2_kind, j2p, desc->j2_n, desc->j2_rcut, desc->j2_cusp_opp,
               j2p ? j2p[0] : 0.0, (j2p && desc->j2_n > 1) ? j2p[1] : 0.0);
  build_radial(P.jas.ei, M > 0 ? desc->j1_kind : QMC_J_NONE, desc->j1_params, desc->j1_n,
               desc->j1_rcut, desc->j1_cusp, 0.0, 0.0);
  if (desc->move_kind == QMC_MOVE_PBYP_DRIFT && !drift_chain_fits(P)) {
    delete s;
    return fail(nullptr, QMC_ERR_ARG, "the particle-by-particle drift chain of this system does not fit one "
                "workgroup's LDS");
  }
  if (s->d.delay_rank > 1 && !delayed_feasible(P, tsize_of(desc->precision), s->d.delay_rank)) {
    delete s;
    return fail(nullptr, QMC_ERR_ARG, "delay_rank %d does not fit one workgroup's LDS for this system",
                desc->delay_rank);
  }
  s->d.ion_pos = s->d.ion_Z = s->d.j2_params = s->d.j1_params = nullptr;
  s->d.arena = nullptr;

  if (desc->j3_gamma) {
    const size_t ng = 2 * (size_t)(desc->j3_m_ei + 1) * (desc->j3_m_ei + 1) * (desc->j3_m_ee + 1);
    std::memcpy(P.j3_g, desc->j3_gamma, ng * sizeof(double));
    P.j3_on = 1;
    P.j3_mei = desc->j3_m_ei;
    P.j3_mee = desc->j3_m_ee;
    P.j3_h = 0.5 * desc->j3_rcut;
  }
  s->d_ions = static_cast<double*>(s->mem.alloc(s->ions4.size() * sizeof(double)));
  if (!s->d_ions) { qmc_destroy_system(s); return fail(nullptr, QMC_ERR_OOM, "device allocation (ions)"); }
  if (hipMemcpyAsync(s->d_ions, s->ions4.data(), s->ions4.size() * sizeof(double), hipMemcpyHostToDevice,
                     s->stream) != hipSuccess) {
    qmc_destroy_system(s);
    return fail(nullptr, QMC_ERR_DEVICE, "ion upload failed");
  }
  P.ions = s->d_ions;
  s->E.enabled = desc->hamiltonian == QMC_H_COULOMB_EWALD;
  if (s->E.enabled) {
    std::vector<double> gvec, sion, htab;
    std::vector<int> segs;
    ewald_setup(s, gvec, sion, segs);
    h_table(htab);
    s->d_gvec = static_cast<double*>(s->mem.alloc(gvec.size() * sizeof(double)));
    s->d_sion = static_cast<double*>(s->mem.alloc(sion.size() * sizeof(double)));
    s->d_segs = static_cast<int*>(s->mem.alloc(segs.size() * sizeof(int)));
    s->d_htab = static_cast<double*>(s->mem.alloc(htab.size() * sizeof(double)));
    if (!s->d_gvec || !s->d_sion || !s->d_segs || !s->d_htab) {
      qmc_destroy_system(s);
      return fail(nullptr, QMC_ERR_OOM, "device allocation (Ewald)");
    }
    if (hipMemcpyAsync(s->d_gvec, gvec.data(), gvec.size() * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_sion, sion.data(), sion.size() * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_segs, segs.data(), segs.size() * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_htab, htab.data(), htab.size() * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess) {
      qmc_destroy_system(s);
      return fail(nullptr, QMC_ERR_DEVICE, "Ewald upload failed");
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) {
      qmc_destroy_system(s);
      return fail(nullptr, QMC_ERR_DEVICE, "stream synchronise failed");
    }
    s->E.gvec = s->d_gvec;
    s->E.s_ion = s->d_sion;
    s->E.segs = s->d_segs;
    s->E.htab = s->d_htab;
  } else if (hipStreamSynchronize(s->stream) != hipSuccess) {
    qmc_destroy_system(s);
    return fail(nullptr, QMC_ERR_DEVICE, "stream synchronise failed");
  }
  s->mark_sys = s->mem.mark();
  s->mark_table = s->mark_sys;
  *out = s;
  return QMC_OK;
}

qmc_status qmc_load_spline_table(qmc_system s, int32_t gx, int32_t gy, int32_t gz, int32_t n_orb,
                                 const void* coefs, int32_t dtype, int32_t coefs_on_device) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (n_orb != s->P.n_orb)
    return fail(s, QMC_ERR_ARG, "n_orb %d must equal max(n_up, n_dn) = %d", n_orb, s->P.n_orb);
  if (gx < 4 || gy < 4 || gz < 4 || (size_t)gx * gy * gz > (size_t)1 << 26)
    return fail(s, QMC_ERR_ARG, "grid sides must be >= 4 (and the grid at most 2^26 points)");
  if (dtype != 4 && dtype != 8) return fail(s, QMC_ERR_ARG, "dtype must be 4 or 8");
  if (!coefs) return fail(s, QMC_ERR_ARG, "coefs is NULL");
  HIP_TRY(s, hipSetDevice(s->device));
  free_walkers(s);
  s->mem.release_to(s->mark_sys);
  s->has_table = false;
  const size_t pts = (size_t)gx * gy * gz;
  const int S = s->P.S;
  const size_t ts = tsize_of(s->d.precision);
  s->d_table = s->mem.alloc(pts * S * ts);
  if (!s->d_table) return fail(s, QMC_ERR_OOM, "device allocation of the %zu-byte table failed", pts * S * ts);
  // Convert/pad on the host: the padded orbital columns are zero.
  const bool same = (size_t)dtype == ts && S == n_orb;
  if (same) {
    HIP_TRY(s, hipMemcpyAsync(s->d_table, coefs, pts * S * ts,
                              coefs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
  } else {
    std::vector<unsigned char> src;
    const unsigned char* hs = static_cast<const unsigned char*>(coefs);
    if (coefs_on_device) {
      src.resize(pts * n_orb * dtype);
      HIP_TRY(s, hipMemcpyAsync(src.data(), coefs, src.size(), hipMemcpyDeviceToHost, s->stream));
      HIP_TRY(s, hipStreamSynchronize(s->stream));
      hs = src.data();
    }
    const size_t chunk = 1 << 16;   // points per staging chunk
    std::vector<unsigned char> stage(chunk * S * ts);
    for (size_t p0 = 0; p0 < pts; p0 += chunk) {
      const size_t np = std::min(chunk, pts - p0);
      std::memset(stage.data(), 0, np * S * ts);
      for (size_t p = 0; p < np; ++p)
        for (int j = 0; j < n_orb; ++j) {
          const size_t si = (p0 + p) * n_orb + j;
          const double v = dtype == 8 ? reinterpret_cast<const double*>(hs)[si]
                                      : (double)reinterpret_cast<const float*>(hs)[si];
          if (ts == 8) reinterpret_cast<double*>(stage.data())[p * S + j] = v;
          else reinterpret_cast<float*>(stage.data())[p * S + j] = (float)v;
        }
      // stream-ordered (a synchronous copy would touch the null stream, which another thread's
      // graph capture must not see); the staging buffer is reused, so each chunk completes first
      HIP_TRY(s, hipMemcpyAsync(static_cast<char*>(s->d_table) + p0 * S * ts, stage.data(), np * S * ts,
                                hipMemcpyHostToDevice, s->stream));
      HIP_TRY(s, hipStreamSynchronize(s->stream));
    }
  }
  s->P.gx = gx;
  s->P.gy = gy;
  s->P.gz = gz;
  s->has_table = true;
  s->mark_table = s->mem.mark();
  return QMC_OK;
}

// sel (nullable): rebuild only the walkers w with sel[w] == sel_value
static qmc_status run_rebuild(qmc_system s, double* drift_dev, const uint32_t* sel = nullptr,
                              uint32_t sel_value = 0) {
  hipError_t e;
  if (s->d.precision == QMC_MIXED)
    e = timed(s, 3, [&] { return launch_rebuild<float>(s->P, walkers_of<float>(s), s->scratch, drift_dev, s->stream, sel, sel_value); });
  else
    e = timed(s, 3, [&] { return launch_rebuild<double>(s->P, walkers_of<double>(s), s->scratch, drift_dev, s->stream, sel, sel_value); });
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "inverse rebuild launch: %s", hipGetErrorString(e));
  return QMC_OK;
}

// Mixed precision: the check of the walkers' inverses (FP64 fallback or early FP64 rebuild),
// on stream st.  after_rebuild: every walker was just rebuilt in FP64 (check all of them);
// otherwise a refinement has just measured every FP32 walker's inverse error: walkers past
// kEtaRebuild are rebuilt, fallback walkers are checked, and walkers back in FP32 are refined.
static hipError_t fallback_check(qmc_system s, hipStream_t st, bool after_rebuild) {
  if (!uses_fallback(s)) return hipSuccess;
  const Walkers<float> wk = walkers_of<float>(s);
  hipError_t e = launch_fb_mark(s->P.W, s->eta, s->fb, s->fbmark, after_rebuild ? 1 : 0, st);
  // on the side stream of pipelined steps the check runs beside the next sweep's gather
  const bool beside = s->side && st == s->side;
  if (e == hipSuccess && !after_rebuild)
    e = launch_rebuild<float>(s->P, wk, s->scratch, nullptr, st, s->fbmark, 1u, beside);
  if (e == hipSuccess) e = launch_fb_residual(s->P, wk, s->scratch, s->fbmark, st);
  if (e == hipSuccess) e = launch_fb_decide(s->P, wk, s->fbmark, after_rebuild ? 0 : 1, st);
  if (e == hipSuccess && !after_rebuild) e = launch_fb_adopt(s->P, wk, s->fbmark, st);
  return e;
}

// Mixed precision: the sweep of the FP64 fallback walkers (the FP32 chain skipped them), in
// FP64 on their FP64 value rows and inverses; any delay rank gives the same decisions.
static hipError_t fallback_chain(qmc_system s, hipStream_t st) {
  if (!uses_fallback(s)) return hipSuccess;
  const Walkers<double> fw = fallback_of(s);
  int K = s->d.delay_rank >= 4 ? std::min(s->d.delay_rank, 16) : 1;
  while (K >= 4 && !delayed_feasible(s->P, sizeof(double), K)) K >>= 1;
  return K >= 4 ? launch_chain_delayed<double>(s->P, fw, K, s->use_mfma, st) : launch_chain<double>(s->P, fw, st);
}

static qmc_status check_singular(qmc_system s) {
  std::vector<int> st(s->P.W);
  HIP_TRY(s, hipMemcpyAsync(st.data(), s->status, st.size() * sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  for (int w = 0; w < s->P.W; ++w)
    if (st[w]) return fail(s, QMC_ERR_SINGULAR, "walker %d: singular Slater matrix (spin mask %d)", w, st[w]);
  return QMC_OK;
}

qmc_status qmc_init_walkers(qmc_system s, int32_t n_walkers, const double* pos) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_table) return fail(s, QMC_ERR_STATE, "load the spline table before init_walkers");
  if (n_walkers < 1 || n_walkers > (1 << 20)) return fail(s, QMC_ERR_ARG, "n_walkers must be in [1, 2^20]");
  HIP_TRY(s, hipSetDevice(s->device));
  free_walkers(s);
  const int W = n_walkers;
  const WalkerSizes z = walker_sizes(s->P.n_up, s->P.n_dn, s->d.precision, W, s->P.n_orb, s->d.move_kind);
  s->pos = static_cast<double*>(s->mem.alloc(z.pos));
  s->prop = static_cast<double*>(s->mem.alloc(z.prop));
  s->vgl = s->mem.alloc(z.vgl);
  s->cur = static_cast<uint8_t*>(s->mem.alloc(z.cur));
  s->binv = s->mem.alloc(z.binv);
  s->logdet = static_cast<double*>(s->mem.alloc(z.logdet));
  s->sign = static_cast<int*>(s->mem.alloc(z.sign));
  s->acc = static_cast<uint8_t*>(s->mem.alloc(z.acc));
  s->nacc = static_cast<uint32_t*>(s->mem.alloc(z.nacc));
  s->status = static_cast<int*>(s->mem.alloc(z.status));
  s->scratch = static_cast<double*>(s->mem.alloc(z.scratch));
  s->drift = static_cast<double*>(s->mem.alloc(z.drift));
  s->energy = static_cast<double*>(s->mem.alloc(z.energy));
  s->nguard = static_cast<uint32_t*>(s->mem.alloc(z.nguard));
  s->sweep_ctr = static_cast<uint32_t*>(s->mem.alloc(z.sweep));
  if (s->d.precision == QMC_MIXED) {
    s->val64 = static_cast<double*>(s->mem.alloc(z.val64));
    s->xinv = s->mem.alloc(z.xinv);
  }
  if (z.binv64) s->binv64 = static_cast<double*>(s->mem.alloc(z.binv64));
  if (z.gitem) {
    s->gorder.key = static_cast<int*>(s->mem.alloc(z.gitem));
    s->gorder.order = static_cast<int*>(s->mem.alloc(z.gitem));
    s->gorder.hist = static_cast<int*>(s->mem.alloc(z.gbucket));
    s->gorder.offs = static_cast<int*>(s->mem.alloc(z.gbucket));
    const int g[3] = {s->P.gx, s->P.gy, s->P.gz};
    for (int a = 0; a < 3; ++a) s->gorder.tile[a] = (g[a] + 15) / 16;   // at most 16 tiles per axis
    const char* e = getenv("QMC_GATHER_ORDER");
    s->gather_ordered = !(e && e[0] == '0');
  }
  if (z.grad64) {
    s->grad64 = static_cast<double*>(s->mem.alloc(z.grad64));
    s->ae_binv64 = static_cast<double*>(s->mem.alloc(z.ae_binv64));
  }
  if (z.fb) {
    s->fb = static_cast<int*>(s->mem.alloc(z.fb));
    s->eta = static_cast<double*>(s->mem.alloc(z.eta));
    s->ecol = static_cast<float*>(s->mem.alloc(z.ecol));
    s->eta_age = static_cast<uint32_t*>(s->mem.alloc(z.eta_age));
    s->pstat = static_cast<uint32_t*>(s->mem.alloc(z.pstat));
    s->fbmark = static_cast<uint32_t*>(s->mem.alloc(z.fbmark));
  }
  const bool ae = s->d.move_kind != QMC_MOVE_PBYP;
  const bool drift = s->d.move_kind == QMC_MOVE_ALL_DRIFT;
  if (drift) {
    s->ae_vcur = static_cast<double*>(s->mem.alloc(z.ae_vel));
    s->ae_vprop = static_cast<double*>(s->mem.alloc(z.ae_vel));
    s->ae_logT = static_cast<double*>(s->mem.alloc(z.ae_logT));
  }
  if (ae) {
    s->ae_binv = s->mem.alloc(z.ae_binv);
    s->ae_logdet = static_cast<double*>(s->mem.alloc(z.ae_logdet));
    s->ae_dj = static_cast<double*>(s->mem.alloc(z.ae_dj));
    s->ae_sign = static_cast<int*>(s->mem.alloc(z.ae_sign));
    s->ae_status = static_cast<int*>(s->mem.alloc(z.ae_status));
  }
  if (!s->pos || !s->prop || !s->vgl || !s->cur || !s->binv || !s->logdet || !s->sign || !s->acc ||
      (z.gitem && (!s->gorder.key || !s->gorder.order || !s->gorder.hist || !s->gorder.offs)) ||
      !s->nacc || !s->status || !s->scratch || !s->drift || !s->energy || !s->nguard || !s->sweep_ctr ||
      (s->d.precision == QMC_MIXED && (!s->val64 || !s->xinv)) ||
      (z.binv64 && !s->binv64) || (z.grad64 && (!s->grad64 || !s->ae_binv64)) ||
      (z.fb && (!s->fb || !s->eta || !s->ecol || !s->eta_age || !s->pstat || !s->fbmark)) ||
      (ae && (!s->ae_binv || !s->ae_logdet || !s->ae_dj || !s->ae_sign || !s->ae_status)) ||
      (drift && (!s->ae_vcur || !s->ae_vprop || !s->ae_logT))) {
    free_walkers(s);
    return fail(s, QMC_ERR_OOM, "device allocation of %zu walker bytes failed", z.total());
  }
  s->P.W = W;
  const size_t N = s->P.N;
  if (pos) {
    std::vector<double> wp((size_t)W * N * 3);
    for (size_t q = 0; q < wp.size(); ++q) {
      const double x = pos[q];
      if (!std::isfinite(x)) { free_walkers(s); return fail(s, QMC_ERR_ARG, "non-finite position"); }
      double y = x - s->d.L * std::floor(x / s->d.L);
      wp[q] = (y >= s->d.L) ? 0.0 : y;
    }
    HIP_TRY(s, hipMemcpyAsync(s->pos, wp.data(), wp.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
  }
  HIP_TRY(s, hipMemsetAsync(s->nguard, 0, z.nguard, s->stream));
  HIP_TRY(s, hipMemsetAsync(s->sweep_ctr, 0, z.sweep, s->stream));
  HIP_TRY(s, hipMemsetAsync(s->acc, 0, z.acc, s->stream));
  HIP_TRY(s, hipMemsetAsync(s->logdet, 0, z.logdet, s->stream));
  HIP_TRY(s, hipMemsetAsync(s->status, 0, z.status, s->stream));
  if (z.gbucket) HIP_TRY(s, hipMemsetAsync(s->gorder.hist, 0, z.gbucket, s->stream));
  if (z.fb) {
    HIP_TRY(s, hipMemsetAsync(s->fb, 0, z.fb, s->stream));
    HIP_TRY(s, hipMemsetAsync(s->pstat, 0, z.pstat, s->stream));
  }
  // Without given positions every electron starts uniform in the cell (INIT stream).  Then the
  // rows, inverses and log|D| of the current positions.
  if (!pos) HIP_TRY(s, launch_init_positions(s->P, s->pos, s->stream));
  hipError_t e;
  if (s->d.precision == QMC_MIXED)
    e = timed(s, 0, [&] { return launch_gather<float>(s->P, walkers_of<float>(s), static_cast<const float*>(s->d_table), 1, s->stream); });
  else
    e = timed(s, 0, [&] { return launch_gather<double>(s->P, walkers_of<double>(s), static_cast<const double*>(s->d_table), 1, s->stream); });
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "orbital gather launch: %s", hipGetErrorString(e));
  qmc_status rst = run_rebuild(s, nullptr);
  if (rst != QMC_OK) return rst;
  e = fallback_check(s, s->stream, true);
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "inverse check launch: %s", hipGetErrorString(e));
  qmc_status st = check_singular(s);
  s->sweep_index = 0;
  s->has_walkers = (st == QMC_OK);
  return st;
}

}  // extern "C"

namespace {

// The proposals of one sweep (gather), on stream st.
qmc_status sweep_gather(qmc_system s, hipStream_t st) {
  hipError_t e;
  // particle-by-particle drift moves evaluate each proposal's row inside the chain
  if (s->d.move_kind == QMC_MOVE_PBYP_DRIFT) return QMC_OK;
  if (s->d.move_kind == QMC_MOVE_ALL_DRIFT && !s->vcur_valid) {
    // drift velocities at the current configuration, which the proposals are centred on
    // (timed with the move kernels, so the gather's own time stays separate).  Afterwards a
    // move keeps them current: an accepted walker takes the velocities computed at R' (the
    // same kernel on the same positions, rows and inverses, so the same bits), a rejected one
    // keeps its own; DMC copies carry them along.
    e = s->d.precision == QMC_MIXED
            ? timed(s, 1, [&] { return launch_ae_velocity<float>(s->P, walkers_of<float>(s), AeProposal<float>{}, 0, s->ae_vcur, nullptr, st); }, st)
            : timed(s, 1, [&] { return launch_ae_velocity<double>(s->P, walkers_of<double>(s), AeProposal<double>{}, 0, s->ae_vcur, nullptr, st); }, st);
    if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "drift velocity launch: %s", hipGetErrorString(e));
    s->vcur_valid = true;
  }
  const GatherOrder* go = s->gather_ordered ? &s->gorder : nullptr;
  if (s->d.precision == QMC_MIXED)
    e = timed(s, 0, [&] { return launch_gather<float>(s->P, walkers_of<float>(s), static_cast<const float*>(s->d_table), 0, st, s->gather_lanes_log2, nullptr, 0, go); }, st);
  else
    e = timed(s, 0, [&] { return launch_gather<double>(s->P, walkers_of<double>(s), static_cast<const double*>(s->d_table), 0, st, s->gather_lanes_log2, nullptr, 0, go); }, st);
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "sweep launch: %s", hipGetErrorString(e));
  return QMC_OK;
}

// The move chain of one sweep and the periodic rebuild when due, on the handle's stream.
// One all-electron move per walker (the sweep's gather already holds R' and its rows): the
// Jastrow change, FP64 determinants of the proposed matrices, then decision and installation.
template <typename T>
hipError_t ae_step(qmc_system s) {
  hipError_t e = launch_ae_jastrow(s->P, s->pos, s->prop, s->ae_dj, s->ae_status, s->stream);
  if (e != hipSuccess) return e;
  Walkers<T> prop = walkers_of<T>(s);
  prop.binv = static_cast<T*>(s->ae_binv);
  prop.logdet = s->ae_logdet;
  prop.sign = s->ae_sign;
  prop.status = s->ae_status;
  prop.row_flip = 1;
  prop.binv64 = s->ae_binv64;   // mixed precision, drift moves: the FP64 inverses at R'
  e = launch_rebuild<T>(s->P, prop, s->scratch, nullptr, s->stream);
  if (e != hipSuccess) return e;
  const bool drift = s->d.move_kind == QMC_MOVE_ALL_DRIFT;
  AeProposal<T> A{static_cast<T*>(s->ae_binv), s->ae_logdet, s->ae_sign, s->ae_status, s->ae_dj, s->ae_logT,
                  velocity_parts(s->P.N), jastrow_parts(s->P.N), s->fixed_node ? 1 : 0,
                  s->fixed_node ? s->dmc_i : nullptr,
                  drift ? s->ae_vprop : nullptr, drift ? s->ae_vcur : nullptr, s->ae_binv64};
  if (s->d.move_kind == QMC_MOVE_ALL_DRIFT) {
    e = launch_ae_velocity<T>(s->P, walkers_of<T>(s), A, 1, s->ae_vprop, s->ae_vcur, s->stream);
    if (e != hipSuccess) return e;
  }
  return launch_ae_apply<T>(s->P, walkers_of<T>(s), A, s->stream);
}

qmc_status sweep_chain(qmc_system s) {
  if (s->d.move_kind == QMC_MOVE_PBYP_DRIFT) {
    const hipError_t e = timed(s, 1, [&] {
      return launch_chain_drift(s->P, walkers_of<double>(s), static_cast<const double*>(s->d_table), s->sweep_index,
                                s->fixed_node ? 1 : 0, s->fixed_node ? s->dmc_i : nullptr, s->stream);
    });
    if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "drift sweep launch: %s", hipGetErrorString(e));
    s->sweep_index += 1;
    if (s->d.recompute_period > 0 && s->sweep_index % (uint32_t)s->d.recompute_period == 0)
      return run_rebuild(s, nullptr);
    return QMC_OK;
  }
  if (s->d.move_kind != QMC_MOVE_PBYP) {
    // the inverses are recomputed at every accepted move, so no periodic rebuild is needed
    const hipError_t e = s->d.precision == QMC_MIXED ? timed(s, 1, [&] { return ae_step<float>(s); })
                                                     : timed(s, 1, [&] { return ae_step<double>(s); });
    if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "all-electron move launch: %s", hipGetErrorString(e));
    s->sweep_index += 1;
    return QMC_OK;
  }
  const int K = s->d.delay_rank;
  const int mfma = s->use_mfma;
  hipError_t e;
  if (s->d.precision == QMC_MIXED)
    e = timed(s, 1, [&] {
      const hipError_t e1 = K > 1 ? launch_chain_delayed<float>(s->P, walkers_of<float>(s), K, mfma, s->stream)
                                  : launch_chain<float>(s->P, walkers_of<float>(s), s->stream);
      return e1 != hipSuccess ? e1 : fallback_chain(s, s->stream);
    });
  else
    e = timed(s, 1, [&] {
      return K > 1 ? launch_chain_delayed<double>(s->P, walkers_of<double>(s), K, mfma, s->stream)
                   : launch_chain<double>(s->P, walkers_of<double>(s), s->stream);
    });
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "sweep launch: %s", hipGetErrorString(e));
  s->sweep_index += 1;
  if (s->d.recompute_period > 0 && s->sweep_index % (uint32_t)s->d.recompute_period == 0) {
    qmc_status st = run_rebuild(s, nullptr);
    if (st != QMC_OK) return st;
    e = fallback_check(s, s->stream, true);
    if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "inverse check launch: %s", hipGetErrorString(e));
  }
  return QMC_OK;
}

// Mixed precision: what a measurement needs first, on st: the refinement of every FP32
// walker's inverse (which the chain then continues from) and the conditioning check.
qmc_status measure_prepare(qmc_system s, hipStream_t st) {
  if (s->d.precision != QMC_MIXED) return QMC_OK;
  const hipError_t e = timed(s, 2, [&] {
    hipError_t er = launch_refine<float>(s->P, walkers_of<float>(s), s->scratch, st);
    return er == hipSuccess ? fallback_check(s, st, false) : er;
  }, st);
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "refinement launch: %s", hipGetErrorString(e));
  return QMC_OK;
}

// The local energies into device memory dst, on st (prepared: measure_prepare has run).
qmc_status measure_prepared(qmc_system s, double* dst, hipStream_t st) {
  hipError_t e;
  if (s->d.precision == QMC_MIXED)
    e = timed(s, 2, [&] { return launch_measure<float>(s->P, walkers_of<float>(s), s->E, s->energy + 4 * (size_t)s->P.W, dst, st); }, st);
  else
    e = timed(s, 2, [&] { return launch_measure<double>(s->P, walkers_of<double>(s), s->E, s->energy + 4 * (size_t)s->P.W, dst, st); }, st);
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "measure launch: %s", hipGetErrorString(e));
  return QMC_OK;
}

// The local energies (with the mixed path's refinement first) into device memory dst, on st.
qmc_status measure_on(qmc_system s, double* dst, hipStream_t st) {
  const qmc_status r = measure_prepare(s, st);
  return r != QMC_OK ? r : measure_prepared(s, dst, st);
}

}  // namespace

extern "C" {

qmc_status qmc_sweep(qmc_system s, int32_t n_sweeps, uint64_t* n_accepted_out) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (n_sweeps < 0) return fail(s, QMC_ERR_ARG, "n_sweeps must be >= 0");
  HIP_TRY(s, hipSetDevice(s->device));
  uint64_t total = 0;
  std::vector<uint32_t> na;
  for (int it = 0; it < n_sweeps; ++it) {
    qmc_status st = sweep_gather(s, s->stream);
    if (st == QMC_OK) st = sweep_chain(s);
    if (st != QMC_OK) return st;
    if (n_accepted_out) {
      na.resize(s->P.W);
      HIP_TRY(s, hipMemcpyAsync(na.data(), s->nacc, na.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
      HIP_TRY(s, hipStreamSynchronize(s->stream));
      for (uint32_t v : na) total += v;
    }
  }
  if (n_accepted_out) *n_accepted_out = total;
  return QMC_OK;
}

qmc_status qmc_measure_local_energy(qmc_system s, double* out, int32_t out_on_device) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (!out) return fail(s, QMC_ERR_ARG, "out is NULL");
  HIP_TRY(s, hipSetDevice(s->device));
  double* dst = out_on_device ? out : s->energy;
  qmc_status st = measure_on(s, dst, s->stream);
  if (st != QMC_OK) return st;
  if (out_on_device) return QMC_OK;
  const size_t nb = (size_t)s->P.W * 4 * sizeof(double);
  HIP_TRY(s, hipMemcpyAsync(out, s->energy, nb, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  for (size_t q = 0; q < (size_t)s->P.W * 4; ++q)
    if (!std::isfinite(out[q])) return fail(s, QMC_ERR_NUMERIC, "non-finite local energy (walker %zu)", q / 4);
  return QMC_OK;
}

qmc_status qmc_run_steps(qmc_system s, int32_t n_steps, double* energies_dev) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (n_steps < 0) return fail(s, QMC_ERR_ARG, "n_steps must be >= 0");
  if (n_steps > 0 && !energies_dev) return fail(s, QMC_ERR_ARG, "energies_dev is NULL");
  if (n_steps == 0) return QMC_OK;
  HIP_TRY(s, hipSetDevice(s->device));
  if (!s->side) {
    HIP_TRY(s, hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
    HIP_TRY(s, hipEventCreateWithFlags(&s->ev_swept, hipEventDisableTiming));
    HIP_TRY(s, hipEventCreateWithFlags(&s->ev_measured, hipEventDisableTiming));
  }
  const size_t stride = (size_t)s->P.W * 4;
  // Step k's measurement reads the positions, current rows and inverses its sweep left; the
  // next sweep's gather writes only the proposals and the other row buffers, so it runs on the
  // handle's stream while the measurement runs on the side stream.  The next chain, which
  // changes what the measurement reads, waits for it.  The mixed path's refinement and
  // conditioning check (which the next chain reads too) run on the handle's stream before the
  // fork: alone they take a third of the time they take beside the gather.
  qmc_status st = sweep_gather(s, s->stream);
  for (int it = 0; it < n_steps && st == QMC_OK; ++it) {
    if (it > 0) HIP_TRY(s, hipStreamWaitEvent(s->stream, s->ev_measured, 0));
    st = sweep_chain(s);
    if (st == QMC_OK) st = measure_prepare(s, s->stream);
    if (st != QMC_OK) break;
    HIP_TRY(s, hipEventRecord(s->ev_swept, s->stream));
    HIP_TRY(s, hipStreamWaitEvent(s->side, s->ev_swept, 0));
    st = measure_prepared(s, energies_dev + (size_t)it * stride, s->side);
    if (st != QMC_OK) break;
    HIP_TRY(s, hipEventRecord(s->ev_measured, s->side));
    if (it + 1 < n_steps) st = sweep_gather(s, s->stream);
  }
  // everything, including the last measurement, completes in the handle's stream order
  HIP_TRY(s, hipStreamWaitEvent(s->stream, s->ev_measured, 0));
  return st;
}

}  // extern "C"

namespace {

DmcState dmc_state_of(qmc_system s, double* stats) {
  const size_t W = s->P.W;
  DmcState D;
  D.w = s->dmc_w;
  D.E = s->dmc_E;
  D.e4 = s->dmc_e4;
  D.wb = s->dmc_wb;
  D.crossed = s->dmc_i;
  D.mult = s->dmc_i + W;
  D.plan = s->dmc_i + 2 * W;
  D.xscan = s->dmc_i + 3 * W;
  D.fscan = s->dmc_i + 4 * W;
  D.ictl = s->dmc_i + 5 * W;
  D.ctl = s->dmc_ctl;
  D.stats = stats;
  D.vel = s->d.move_kind == QMC_MOVE_ALL_DRIFT ? s->ae_vcur : nullptr;
  return D;
}

}  // namespace

extern "C" {

qmc_status qmc_dmc_init(qmc_system s, int32_t n_target, double e_trial, double feedback) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (s->d.move_kind != QMC_MOVE_ALL_DRIFT && s->d.move_kind != QMC_MOVE_PBYP_DRIFT)
    return fail(s, QMC_ERR_STATE, "diffusion Monte Carlo needs drift moves (QMC_MOVE_ALL_DRIFT or "
                "QMC_MOVE_PBYP_DRIFT)");
  const int W = s->P.W;
  if (n_target < 1 || n_target > W) return fail(s, QMC_ERR_ARG, "n_target must be in [1, %d]", W);
  if (!(feedback >= 0.0) || !std::isfinite(feedback)) return fail(s, QMC_ERR_ARG, "feedback must be >= 0");
  if (!std::isnan(e_trial) && !std::isfinite(e_trial)) return fail(s, QMC_ERR_ARG, "e_trial must be finite or NaN");
  HIP_TRY(s, hipSetDevice(s->device));
  if (!s->dmc_w) {
    s->dmc_w = static_cast<double*>(s->mem.alloc(W * sizeof(double)));
    s->dmc_E = static_cast<double*>(s->mem.alloc(W * sizeof(double)));
    s->dmc_e4 = static_cast<double*>(s->mem.alloc(W * 4 * sizeof(double)));
    s->dmc_wb = static_cast<double*>(s->mem.alloc(W * 2 * sizeof(double)));
    s->dmc_ctl = static_cast<double*>(s->mem.alloc(2 * sizeof(double)));
    s->dmc_i = static_cast<int*>(s->mem.alloc((5 * (size_t)W + 3) * sizeof(int)));
    if (!s->dmc_w || !s->dmc_E || !s->dmc_e4 || !s->dmc_wb || !s->dmc_ctl || !s->dmc_i)
      return fail(s, QMC_ERR_OOM, "device allocation of the DMC population failed");
  }
  // local energies of every slot's configuration; the first n_target slots are alive
  qmc_status st = measure_on(s, s->dmc_e4, s->stream);
  if (st != QMC_OK) return st;
  std::vector<double> e4((size_t)W * 4), E(W), w(W);
  HIP_TRY(s, hipMemcpyAsync(e4.data(), s->dmc_e4, e4.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  double se = 0.0;
  for (int j = 0; j < W; ++j) {
    E[j] = e4[4 * j] + e4[4 * j + 1] + e4[4 * j + 2] + e4[4 * j + 3];
    w[j] = j < n_target ? 1.0 : 0.0;
    if (j < n_target) {
      if (!std::isfinite(E[j])) return fail(s, QMC_ERR_NUMERIC, "non-finite local energy (walker %d)", j);
      se += E[j];
    }
  }
  const double ctl[2] = {std::isnan(e_trial) ? se / n_target : e_trial, feedback};
  const int ictl[3] = {0, 0, n_target};
  HIP_TRY(s, hipMemcpyAsync(s->dmc_E, E.data(), W * sizeof(double), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(s, hipMemcpyAsync(s->dmc_w, w.data(), W * sizeof(double), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(s, hipMemcpyAsync(s->dmc_ctl, ctl, sizeof ctl, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(s, hipMemcpyAsync(s->dmc_i + 5 * (size_t)W, ictl, sizeof ictl, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  s->dmc_ready = true;
  return QMC_OK;
}

qmc_status qmc_dmc_steps(qmc_system s, int32_t n_steps, double* stats_dev) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers || !s->dmc_ready) return fail(s, QMC_ERR_STATE, "qmc_dmc_init first");
  if (n_steps < 0) return fail(s, QMC_ERR_ARG, "n_steps must be >= 0");
  if (n_steps > 0 && !stats_dev) return fail(s, QMC_ERR_ARG, "stats_dev is NULL");
  HIP_TRY(s, hipSetDevice(s->device));
  qmc_status st = QMC_OK;
  s->fixed_node = true;
  for (int k = 0; k < n_steps && st == QMC_OK; ++k) {
    st = sweep_gather(s, s->stream);
    if (st == QMC_OK) st = sweep_chain(s);
    if (st == QMC_OK) st = measure_on(s, s->dmc_e4, s->stream);
    if (st != QMC_OK) break;
    const DmcState D = dmc_state_of(s, stats_dev + 6 * (size_t)k);
    hipError_t e = timed(s, 3, [&] { return launch_dmc_branch(s->P, D, s->stream); });
    if (e == hipSuccess)
      e = timed(s, 3, [&] {
        return s->d.precision == QMC_MIXED ? launch_dmc_copy<float>(s->P, walkers_of<float>(s), D, s->stream)
                                           : launch_dmc_copy<double>(s->P, walkers_of<double>(s), D, s->stream);
      });
    if (e != hipSuccess) st = fail(s, QMC_ERR_DEVICE, "branching launch: %s", hipGetErrorString(e));
  }
  s->fixed_node = false;
  return st;
}

qmc_status qmc_dmc_get(qmc_system s, double* weights, double* energies, double* e_trial, int32_t* population) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers || !s->dmc_ready) return fail(s, QMC_ERR_STATE, "qmc_dmc_init first");
  HIP_TRY(s, hipSetDevice(s->device));
  const int W = s->P.W;
  std::vector<double> w(W), ctl(2);
  int ictl[3];
  HIP_TRY(s, hipMemcpyAsync(w.data(), s->dmc_w, W * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (energies) HIP_TRY(s, hipMemcpyAsync(energies, s->dmc_E, W * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipMemcpyAsync(ctl.data(), s->dmc_ctl, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipMemcpyAsync(ictl, s->dmc_i + 5 * (size_t)W, sizeof ictl, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  int pop = 0;
  for (double v : w) pop += v > 0.0;
  if (weights) std::memcpy(weights, w.data(), W * sizeof(double));
  if (e_trial) *e_trial = ctl[0];
  if (population) *population = pop;
  if (ictl[1]) return fail(s, QMC_ERR_NUMERIC, "the population died out");
  return QMC_OK;
}

qmc_status qmc_dmc_get_branching(qmc_system s, double* weights, double* energies, int32_t* mult, int32_t* plan) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers || !s->dmc_ready) return fail(s, QMC_ERR_STATE, "qmc_dmc_init first");
  HIP_TRY(s, hipSetDevice(s->device));
  const size_t W = s->P.W;
  int ictl[3];
  HIP_TRY(s, hipMemcpyAsync(ictl, s->dmc_i + 5 * W, sizeof ictl, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  if (ictl[0] == 0) return fail(s, QMC_ERR_STATE, "no DMC step has run since qmc_dmc_init");
  std::vector<double> wb(2 * W);
  HIP_TRY(s, hipMemcpyAsync(wb.data(), s->dmc_wb, wb.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (mult) HIP_TRY(s, hipMemcpyAsync(mult, s->dmc_i + W, W * sizeof(int), hipMemcpyDeviceToHost, s->stream));
  if (plan) HIP_TRY(s, hipMemcpyAsync(plan, s->dmc_i + 2 * W, W * sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  for (size_t j = 0; j < W; ++j) {
    if (weights) weights[j] = wb[2 * j];
    if (energies) energies[j] = wb[2 * j + 1];
  }
  return QMC_OK;
}

qmc_status qmc_get_walkers(qmc_system s, double* pos, double* logabs_det, int32_t* sign) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  HIP_TRY(s, hipSetDevice(s->device));
  const size_t W = s->P.W, N = s->P.N;
  if (pos) HIP_TRY(s, hipMemcpyAsync(pos, s->pos, W * N * 3 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (logabs_det) HIP_TRY(s, hipMemcpyAsync(logabs_det, s->logdet, W * 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (sign) HIP_TRY(s, hipMemcpyAsync(sign, s->sign, W * 2 * sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return QMC_OK;
}

qmc_status qmc_get_accept_log(qmc_system s, uint8_t* bits) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (!bits) return fail(s, QMC_ERR_ARG, "bits is NULL");
  HIP_TRY(s, hipSetDevice(s->device));
  HIP_TRY(s, hipMemcpyAsync(bits, s->acc, (size_t)s->P.W * s->P.N, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return QMC_OK;
}

qmc_status qmc_get_counters(qmc_system s, uint64_t* redecided, uint64_t* sweeps) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  HIP_TRY(s, hipSetDevice(s->device));
  if (redecided) {
    std::vector<uint32_t> g(s->P.W);
    HIP_TRY(s, hipMemcpyAsync(g.data(), s->nguard, g.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    uint64_t t = 0;
    for (uint32_t v : g) t += v;
    *redecided = t;
  }
  if (sweeps) *sweeps = s->sweep_index;
  return QMC_OK;
}

qmc_status qmc_set_sweep_index(qmc_system s, uint64_t sweep_index) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (sweep_index > 0xFFFFFFFFull) return fail(s, QMC_ERR_ARG, "sweep_index must be below 2^32");
  HIP_TRY(s, hipSetDevice(s->device));
  const uint32_t v = (uint32_t)sweep_index;
  // the device counter is what the gathers read (and graph replays advance)
  HIP_TRY(s, hipMemcpyAsync(s->sweep_ctr, &v, sizeof v, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  s->sweep_index = v;
  return QMC_OK;
}

qmc_status qmc_get_precision_stats(qmc_system s, uint64_t* early_rebuilds, uint64_t* fallback_sweeps,
                                   int32_t* fallback_now, int32_t* fallback_mask) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  HIP_TRY(s, hipSetDevice(s->device));
  const int W = s->P.W;
  std::vector<uint32_t> ps(2 * (size_t)W, 0u);
  std::vector<int> fb(W, 0);
  if (uses_fallback(s)) {
    HIP_TRY(s, hipMemcpyAsync(ps.data(), s->pstat, ps.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipMemcpyAsync(fb.data(), s->fb, fb.size() * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
  }
  uint64_t rb = 0, fs = 0;
  int32_t now = 0;
  for (int w = 0; w < W; ++w) {
    rb += ps[2 * (size_t)w];
    fs += ps[2 * (size_t)w + 1];
    now += fb[w] ? 1 : 0;
    if (fallback_mask) fallback_mask[w] = fb[w] ? 1 : 0;
  }
  if (early_rebuilds) *early_rebuilds = rb;
  if (fallback_sweeps) *fallback_sweeps = fs;
  if (fallback_now) *fallback_now = now;
  return QMC_OK;
}

qmc_status qmc_recompute(qmc_system s, double* drift_out) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  HIP_TRY(s, hipSetDevice(s->device));
  HIP_TRY(s, hipMemsetAsync(s->status, 0, (size_t)s->P.W * sizeof(int), s->stream));
  qmc_status st = run_rebuild(s, s->drift);
  if (st != QMC_OK) return st;
  const hipError_t e = fallback_check(s, s->stream, true);
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "inverse check launch: %s", hipGetErrorString(e));
  s->vcur_valid = false;   // (the same bits would come back; recomputed for simplicity)
  if (drift_out)
    HIP_TRY(s, hipMemcpyAsync(drift_out, s->drift, (size_t)s->P.W * 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  return check_singular(s);
}

}  // extern "C"

namespace {

// Staging of qmc_eval_spo_vgl_noalloc: a fixed array in every GPU's memory, held until the
// process ends.  In host code the name stands for nothing usable: the device address of each
// GPU's copy is taken once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to copies and kernels.
static __device__ __align__(256) double scratch[QMC_NOALLOC_DOUBLES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of scratch (looked up on the first call per device), or null with *e set.
double* scratch_on(int device, hipError_t* e) {
  *e = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *e = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    *e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*e != hipSuccess || !ptr) {
      if (*e == hipSuccess) *e = hipErrorInvalidSymbol;
      return nullptr;
    }
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

qmc_status qmc_eval_spo_vgl_noalloc(qmc_system s, int32_t n, const double* pos, double* out) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_table) return fail(s, QMC_ERR_STATE, "load the spline table first");
  if (n < 0 || (n > 0 && (!pos || !out))) return fail(s, QMC_ERR_ARG, "bad arguments");
  if (n == 0) return QMC_OK;
  const size_t need = (size_t)n * (3 + (size_t)kComp * s->P.n_orb);
  if (need > (size_t)QMC_NOALLOC_DOUBLES)
    return fail(s, QMC_ERR_ARG, "%d points of %d orbitals need %zu doubles of staging, more than the %d the "
                "fixed array holds", n, s->P.n_orb, need, (int)QMC_NOALLOC_DOUBLES);
  HIP_TRY(s, hipSetDevice(s->device));
  hipError_t e;
  double* base = scratch_on(s->device, &e);
  if (!base) return fail(s, QMC_ERR_DEVICE, "device address of the staging array: %s", hipGetErrorString(e));
  double* dp = base;                       // [n][3] positions
  double* dout = base + (size_t)n * 3;     // [n][5][n_orb] results (every entry written by the kernel)
  const size_t ob = (size_t)n * kComp * s->P.n_orb * sizeof(double);
  e = hipMemcpyAsync(dp, pos, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) {
    if (s->d.precision == QMC_MIXED)
      e = launch_eval_points<float>(s->P, static_cast<const float*>(s->d_table), dp, n, dout, s->stream);
    else
      e = launch_eval_points<double>(s->P, static_cast<const double*>(s->d_table), dp, n, dout, s->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, ob, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "eval_spo_vgl_noalloc: %s", hipGetErrorString(e));
  return QMC_OK;
}

qmc_status qmc_eval_spo_vgl(qmc_system s, int32_t n, const double* pos, double* out) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_table) return fail(s, QMC_ERR_STATE, "load the spline table first");
  if (n < 0 || (n > 0 && (!pos || !out))) return fail(s, QMC_ERR_ARG, "bad arguments");
  if (n == 0) return QMC_OK;
  HIP_TRY(s, hipSetDevice(s->device));
  double *dp = nullptr, *dout = nullptr;
  const size_t ob = (size_t)n * kComp * s->P.n_orb * sizeof(double);
  HIP_TRY(s, hipMalloc(&dp, (size_t)n * 3 * sizeof(double)));
  hipError_t e = hipMalloc(&dout, ob);
  if (e == hipSuccess) e = hipMemcpyAsync(dp, pos, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) {
    if (s->d.precision == QMC_MIXED)
      e = launch_eval_points<float>(s->P, static_cast<const float*>(s->d_table), dp, n, dout, s->stream);
    else
      e = launch_eval_points<double>(s->P, static_cast<const double*>(s->d_table), dp, n, dout, s->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, ob, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(dp);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return fail(s, QMC_ERR_DEVICE, "eval_spo_vgl: %s", hipGetErrorString(e));
  return QMC_OK;
}

qmc_status qmc_set_timing(qmc_system s, int32_t enable) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  s->timing = enable != 0;
  return QMC_OK;
}

qmc_status qmc_kernel_timing(qmc_system s, int32_t kernel_class, double* total_ms, int64_t* launches,
                             int32_t reset) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (kernel_class < 0 || kernel_class > 3) return fail(s, QMC_ERR_ARG, "kernel_class must be 0..3");
  HIP_TRY(s, hipSetDevice(s->device));
  TimerClass& tc = s->timers[kernel_class];
  if (!tc.live.empty()) HIP_TRY(s, hipEventSynchronize(tc.live.back().second));
  for (auto& ev : tc.live) {
    float ms = 0.f;
    HIP_TRY(s, hipEventElapsedTime(&ms, ev.first, ev.second));
    tc.ms += ms;
    tc.launches += 1;
    tc.pool.push_back(ev);
  }
  tc.live.clear();
  if (total_ms) *total_ms = tc.ms;
  if (launches) *launches = tc.launches;
  if (reset) { tc.ms = 0.0; tc.launches = 0; }
  return QMC_OK;
}

qmc_status qmc_set_delay_rank(qmc_system s, int32_t delay_rank) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!valid_rank(delay_rank))
    return fail(s, QMC_ERR_ARG, "delay_rank %d: use 1 or a power of two in [4, 64]", delay_rank);
  if (delay_rank > 1 && !delayed_feasible(s->P, tsize_of(s->d.precision), delay_rank))
    return fail(s, QMC_ERR_ARG, "delay_rank %d does not fit one workgroup's LDS for this system", delay_rank);
  s->d.delay_rank = delay_rank == 0 ? 1 : delay_rank;
  return QMC_OK;
}

qmc_status qmc_set_gather_lanes(qmc_system s, int32_t lanes_log2) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (lanes_log2 < -1 || lanes_log2 > 6) return fail(s, QMC_ERR_ARG, "lanes_log2 must be -1 or 0..6");
  s->gather_lanes_log2 = lanes_log2;
  return QMC_OK;
}

qmc_status qmc_autotune_gather(qmc_system s, int32_t trial_sweeps, int32_t* best_lanes_log2, double* best_ms) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (!s->d_table) return fail(s, QMC_ERR_STATE, "load_spline_table first");
  if (trial_sweeps < 2) return fail(s, QMC_ERR_ARG, "need >= 2 trial sweeps");
  const int V = s->d.precision == QMC_MIXED ? 4 : 2;
  const int base = gather_tpi_log2(s->P.S / V);
  const bool timing_was = s->timing;
  const int was = s->gather_lanes_log2;
  s->timing = true;
  int best = -1;
  double best_t = 0.0;
  for (int tl = base - 2; tl <= base + 2; ++tl) {
    if (tl < 0 || tl > 6) continue;
    s->gather_lanes_log2 = tl;
    qmc_status st = qmc_sweep(s, 1, nullptr);   // untimed: first use of this width
    double ms = 0.0;
    int64_t cnt = 0;
    if (st == QMC_OK) st = qmc_kernel_timing(s, 0, nullptr, nullptr, 1);
    if (st == QMC_OK) st = qmc_sweep(s, trial_sweeps - 1, nullptr);
    if (st == QMC_OK) st = qmc_kernel_timing(s, 0, &ms, &cnt, 1);
    if (st != QMC_OK) {
      s->timing = timing_was;
      s->gather_lanes_log2 = was;
      return st;
    }
    const double per = ms / (double)(cnt > 0 ? cnt : 1);
    if (best < 0 || per < best_t) { best = tl; best_t = per; }
  }
  s->gather_lanes_log2 = best;
  s->timing = timing_was;
  if (best_lanes_log2) *best_lanes_log2 = best;
  if (best_ms) *best_ms = best_t;
  return QMC_OK;
}

qmc_status qmc_autotune_delay(qmc_system s, const int32_t* ranks, int32_t n_ranks, int32_t trial_sweeps,
                              int32_t* best_rank, double* best_ms) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (!ranks || n_ranks < 1 || trial_sweeps < 2) return fail(s, QMC_ERR_ARG, "need candidates and >= 2 trial sweeps");
  for (int i = 0; i < n_ranks; ++i)
    if (!valid_rank(ranks[i])) return fail(s, QMC_ERR_ARG, "candidate delay rank %d is not valid", ranks[i]);
  const size_t ts = tsize_of(s->d.precision);
  const bool timing_was = s->timing;
  const int rank_was = s->d.delay_rank;
  s->timing = true;
  int best = -1;
  double best_t = 0.0;
  for (int i = 0; i < n_ranks; ++i) {
    if (ranks[i] > 1 && !delayed_feasible(s->P, ts, ranks[i])) continue;   // does not fit the LDS
    s->d.delay_rank = ranks[i] == 0 ? 1 : ranks[i];
    qmc_status st = qmc_sweep(s, 1, nullptr);   // untimed: first use of this variant
    double ms = 0.0;
    int64_t cnt = 0;
    if (st == QMC_OK) st = qmc_kernel_timing(s, 1, nullptr, nullptr, 1);
    if (st == QMC_OK) st = qmc_sweep(s, trial_sweeps - 1, nullptr);
    if (st == QMC_OK) st = qmc_kernel_timing(s, 1, &ms, &cnt, 1);
    if (st != QMC_OK) {
      s->timing = timing_was;
      s->d.delay_rank = rank_was;
      return st;
    }
    const double per = ms / (double)(cnt > 0 ? cnt : 1);
    if (best < 0 || per < best_t) { best = s->d.delay_rank; best_t = per; }
  }
  if (best < 0) {
    s->d.delay_rank = rank_was;
    s->timing = timing_was;
    return fail(s, QMC_ERR_ARG, "no candidate delay rank fits this system");
  }
  s->d.delay_rank = best;
  s->timing = timing_was;
  if (best_rank) *best_rank = best;
  if (best_ms) *best_ms = best_t;
  return QMC_OK;
}

qmc_status qmc_get_last_energies(qmc_system s, double* out) {
  if (!s) return fail(nullptr, QMC_ERR_ARG, "handle is NULL");
  if (!s->has_walkers) return fail(s, QMC_ERR_STATE, "init_walkers first");
  if (!out) return fail(s, QMC_ERR_ARG, "out is NULL");
  HIP_TRY(s, hipSetDevice(s->device));
  HIP_TRY(s, hipMemcpyAsync(out, s->energy, (size_t)s->P.W * 4 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return QMC_OK;
}

qmc_status qmc_destroy_system(qmc_system s) {
  if (!s) return QMC_OK;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  if (s->side) {
    (void)hipStreamSynchronize(s->side);
    (void)hipStreamDestroy(s->side);
    (void)hipEventDestroy(s->ev_swept);
    (void)hipEventDestroy(s->ev_measured);
  }
  for (auto& tc : s->timers) {
    for (auto& ev : tc.live) { (void)hipEventDestroy(ev.first); (void)hipEventDestroy(ev.second); }
    for (auto& ev : tc.pool) { (void)hipEventDestroy(ev.first); (void)hipEventDestroy(ev.second); }
  }
  s->mem.release_to(0);
  delete s;
  return QMC_OK;
}

}  // extern "C"

struct qmc_batch_s {
  std::vector<qmc_system> sys;
  hipStream_t stream = nullptr;
  int device = 0, precision = 0;
  std::string err;
  void* d_sysdev = nullptr;
  int2* d_maps = nullptr;
  int2 *gmap = nullptr, *clmap = nullptr, *cgmap = nullptr, *mmap = nullptr, *fmap = nullptr;
  int n_g = 0, n_cl = 0, n_cg = 0, n_m = 0, n_f = 0;
  size_t lds_cl = 0, lds_cg = 0, lds_m = 0;
  int use_mfma = 1;
  bool use_graph = false;
  int graph_fallbacks = 0;   // captures invalidated from outside (the batch then launches eagerly)
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // ordering against the members' own streams: one event per distinct member stream
  // (work queued there before a batch sweep) and one on the batch stream (after it)
  std::vector<hipStream_t> member_streams;
  std::vector<hipEvent_t> member_ev;
  hipEvent_t done_ev = nullptr;
  TimerClass timer;
};

namespace {

qmc_status bfail(qmc_batch b, qmc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  if (b) b->err = buf;
  return st;
}

#define BHIP_TRY(b, expr)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return bfail((b), QMC_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

int max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    return v;
  return 65536;
}

template <typename T>
qmc_status batch_build(qmc_batch b) {
  const int n = (int)b->sys.size();
  const int V = sizeof(T) == sizeof(double) ? 2 : 4;
  const size_t budget = (size_t)max_lds_per_block();
  std::vector<SysDev<T>> sd(n);
  std::vector<int2> g, cl, cg, m, f;
  for (int i = 0; i < n; ++i) {
    qmc_system s = b->sys[i];
    SysDev<T>& d = sd[i];
    std::memset(&d, 0, sizeof d);
    d.P = s->P;
    d.W = walkers_of<T>(s);
    d.E = s->E;
    d.table = static_cast<const T*>(s->d_table);
    d.eout = s->energy;
    d.mpart = s->energy + 4 * (size_t)s->P.W;
    d.np = measure_parts(s->P.W);
    d.scratch = s->scratch;
    d.K = s->d.delay_rank;
    const int nmax = s->P.n_up > s->P.n_dn ? s->P.n_up : s->P.n_dn;
    d.ldl = nmax | 1;
    d.tpi_log2 = s->gather_lanes_log2 >= 0 ? s->gather_lanes_log2 : gather_tpi_log2(s->P.S / V);
    const long items = (long)s->P.W * s->P.N;
    const long per_block = kBlock >> d.tpi_log2;
    for (long it = 0; it < items; it += per_block) g.push_back(make_int2(i, (int)it));
    const size_t extra = sizeof(Jastrow) + sizeof(SysDev<T>);
    const size_t bl = delayed_lds_bytes(s->P, sizeof(T), true, d.K);
    const size_t gl = delayed_lds_bytes(s->P, sizeof(T), false, d.K);
    const bool in_lds = bl + extra <= budget;
    if (!in_lds && gl + extra > budget)
      return bfail(b, QMC_ERR_ARG, "system %d does not fit the batched chain's LDS", i);
    for (int w = 0; w < s->P.W; ++w) {
      (in_lds ? cl : cg).push_back(make_int2(i, w));
      f.push_back(make_int2(i, w));
      for (int p = 0; p < d.np; ++p) m.push_back(make_int2(i, w * d.np + p));
    }
    if (in_lds) b->lds_cl = std::max(b->lds_cl, bl);
    else b->lds_cg = std::max(b->lds_cg, gl);
    b->lds_m = std::max(b->lds_m, measure_lds_bytes(s->P, d.np));
  }
  BHIP_TRY(b, hipMalloc(&b->d_sysdev, sizeof(SysDev<T>) * n));
  const size_t nm = g.size() + cl.size() + cg.size() + m.size() + f.size();
  BHIP_TRY(b, hipMalloc(reinterpret_cast<void**>(&b->d_maps), sizeof(int2) * nm));
  b->gmap = b->d_maps;
  b->clmap = b->gmap + g.size();
  b->cgmap = b->clmap + cl.size();
  b->mmap = b->cgmap + cg.size();
  b->fmap = b->mmap + m.size();
  b->n_g = (int)g.size(); b->n_cl = (int)cl.size(); b->n_cg = (int)cg.size(); b->n_m = (int)m.size();
  b->n_f = (int)f.size();
  std::vector<int2> all;
  all.reserve(nm);
  all.insert(all.end(), g.begin(), g.end());
  all.insert(all.end(), cl.begin(), cl.end());
  all.insert(all.end(), cg.begin(), cg.end());
  all.insert(all.end(), m.begin(), m.end());
  all.insert(all.end(), f.begin(), f.end());
  BHIP_TRY(b, hipMemcpyAsync(b->d_sysdev, sd.data(), sizeof(SysDev<T>) * n, hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->d_maps, all.data(), sizeof(int2) * nm, hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return QMC_OK;
}

// One sweep of every member (gather, chain launches) and, if measure, the fused measurement.
template <typename T>
hipError_t batch_launch(qmc_batch b, int sweep, int measure) {
  const SysDev<T>* sd = static_cast<const SysDev<T>*>(b->d_sysdev);
  hipError_t e = hipSuccess;
  if (sweep) {
    e = launch_gather_batched<T>(sd, b->gmap, b->n_g, b->stream);
    if (e == hipSuccess)
      e = launch_chain_delayed_batched<T>(sd, b->clmap, b->n_cl, true, b->use_mfma, b->lds_cl, b->stream);
    if (e == hipSuccess)
      e = launch_chain_delayed_batched<T>(sd, b->cgmap, b->n_cg, false, b->use_mfma, b->lds_cg, b->stream);
    // mixed precision: each member's FP64 fallback walkers (the fused chains skipped them)
    for (size_t i = 0; e == hipSuccess && i < b->sys.size(); ++i) e = fallback_chain(b->sys[i], b->stream);
  }
  if (e == hipSuccess && measure && b->precision == QMC_MIXED) {
    e = launch_refine_batched<float>(reinterpret_cast<const SysDev<float>*>(sd), b->fmap, b->n_f, b->stream);
    for (size_t i = 0; e == hipSuccess && i < b->sys.size(); ++i) e = fallback_check(b->sys[i], b->stream, false);
  }
  if (e == hipSuccess && measure) e = launch_measure_batched<T>(sd, b->mmap, b->n_m, b->fmap, b->n_f, b->lds_m, b->stream);
  return e;
}

hipError_t batch_launch_any(qmc_batch b, int sweep, int measure) {
  return b->precision == QMC_MIXED ? batch_launch<float>(b, sweep, measure) : batch_launch<double>(b, sweep, measure);
}

}  // namespace

extern "C" {

qmc_status qmc_batch_create(const qmc_system* systems, int32_t n_systems, void* hip_stream, qmc_batch* out) {
  if (!out) return bfail(nullptr, QMC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!systems || n_systems < 1) return bfail(nullptr, QMC_ERR_ARG, "need at least one system");
  qmc_batch b = new (std::nothrow) qmc_batch_s;
  if (!b) return bfail(nullptr, QMC_ERR_OOM, "host allocation failed");
  b->stream = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < n_systems; ++i) {
    qmc_system s = systems[i];
    if (!s || !s->has_walkers) { delete b; return bfail(nullptr, QMC_ERR_STATE, "system %d is not initialised", i); }
    if (i == 0) { b->device = s->device; b->precision = s->d.precision; b->use_mfma = s->use_mfma; }
    if (s->device != b->device || s->d.precision != b->precision) {
      delete b;
      return bfail(nullptr, QMC_ERR_ARG, "systems of a batch share the device and the precision");
    }
    if (s->d.move_kind != QMC_MOVE_PBYP) {
      delete b;
      return bfail(nullptr, QMC_ERR_ARG, "system %d: batches run particle-by-particle moves", i);
    }
    if (s->d.delay_rank < 4) {
      delete b;
      return bfail(nullptr, QMC_ERR_ARG, "system %d: batches run the delayed chain (delay rank >= 4)", i);
    }
    b->sys.push_back(s);
  }
  if (hipSetDevice(b->device) != hipSuccess) { delete b; return bfail(nullptr, QMC_ERR_DEVICE, "hipSetDevice failed"); }
  for (qmc_system s : b->sys)
    if (hipStreamSynchronize(s->stream) != hipSuccess) { delete b; return bfail(nullptr, QMC_ERR_DEVICE, "member stream sync failed"); }
  qmc_status st = b->precision == QMC_MIXED ? batch_build<float>(b) : batch_build<double>(b);
  if (st != QMC_OK) {
    qmc_batch_destroy(b);
    return st;
  }
  for (qmc_system s : b->sys)
    if (s->stream != b->stream &&
        std::find(b->member_streams.begin(), b->member_streams.end(), s->stream) == b->member_streams.end())
      b->member_streams.push_back(s->stream);
  b->member_ev.assign(b->member_streams.size(), nullptr);
  bool ok = hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming) == hipSuccess;
  for (auto& e : b->member_ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    qmc_batch_destroy(b);
    return bfail(nullptr, QMC_ERR_DEVICE, "event creation failed");
  }
  *out = b;
  return QMC_OK;
}

qmc_status qmc_batch_set_graph(qmc_batch b, int32_t use_graph) {
  if (!b) return bfail(nullptr, QMC_ERR_ARG, "batch is NULL");
  if (use_graph && b->stream == nullptr)
    return bfail(b, QMC_ERR_ARG, "graph capture needs a non-default stream");
  b->use_graph = use_graph != 0;
  return QMC_OK;
}

qmc_status qmc_batch_sweep(qmc_batch b, int32_t n_sweeps, int32_t measure) {
  if (!b) return bfail(nullptr, QMC_ERR_ARG, "batch is NULL");
  if (n_sweeps < 0) return bfail(b, QMC_ERR_ARG, "n_sweeps must be >= 0");
  BHIP_TRY(b, hipSetDevice(b->device));
  measure = measure ? 1 : 0;
  // gexec[v]: captured sweep (v = 0) or sweep + measurement (v = 1), made on first use
  auto graph_for = [&](int v) -> qmc_status {
    if (b->gexec[v]) return QMC_OK;
    hipGraph_t graph = nullptr;
    BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
    const hipError_t e = batch_launch_any(b, 1, v);
    const hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
    if (e2 == hipErrorStreamCaptureInvalidated && e == hipSuccess) {
      // the capture was invalidated from outside the batch's launches (another thread's work on
      // the device): nothing captured ran, so this batch goes on with ordinary launches
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      b->use_graph = false;
      b->graph_fallbacks += 1;
      return QMC_OK;
    }
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return bfail(b, QMC_ERR_DEVICE, "sweep capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    const hipError_t e3 = hipGraphInstantiate(&b->gexec[v], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
      b->gexec[v] = nullptr;
      return bfail(b, QMC_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e3));
    }
    return QMC_OK;
  };
  if (n_sweeps == 0) return QMC_OK;
  for (size_t i = 0; i < b->member_streams.size(); ++i) {
    BHIP_TRY(b, hipEventRecord(b->member_ev[i], b->member_streams[i]));
    BHIP_TRY(b, hipStreamWaitEvent(b->stream, b->member_ev[i], 0));
  }
  for (int it = 0; it < n_sweeps; ++it) {
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!b->timer.pool.empty()) { ev = b->timer.pool.back(); b->timer.pool.pop_back(); }
    else {
      BHIP_TRY(b, hipEventCreate(&ev.first));
      BHIP_TRY(b, hipEventCreate(&ev.second));
    }
    // members whose periodic FP64 rebuild falls after this sweep: as in qmc_sweep, the rebuild
    // precedes the measurement, so the sweep runs without it and the measurement follows eagerly
    bool due = false;
    for (qmc_system s : b->sys)
      due |= s->d.recompute_period > 0 && (s->sweep_index + 1) % (uint32_t)s->d.recompute_period == 0;
    const int fused_measure = measure && !due;
    if (b->use_graph) {
      const qmc_status st = graph_for(fused_measure);
      if (st != QMC_OK) return st;
    }
    BHIP_TRY(b, hipEventRecord(ev.first, b->stream));
    if (b->use_graph) {
      BHIP_TRY(b, hipGraphLaunch(b->gexec[fused_measure], b->stream));
    } else {
      BHIP_TRY(b, batch_launch_any(b, 1, fused_measure));
    }
    for (qmc_system s : b->sys) {
      s->sweep_index += 1;
      if (s->d.recompute_period > 0 && s->sweep_index % (uint32_t)s->d.recompute_period == 0) {
        hipError_t e = s->d.precision == QMC_MIXED
            ? launch_rebuild<float>(s->P, walkers_of<float>(s), s->scratch, nullptr, b->stream)
            : launch_rebuild<double>(s->P, walkers_of<double>(s), s->scratch, nullptr, b->stream);
        if (e == hipSuccess) e = fallback_check(s, b->stream, true);
        if (e != hipSuccess) return bfail(b, QMC_ERR_DEVICE, "rebuild launch: %s", hipGetErrorString(e));
      }
    }
    if (measure && due) BHIP_TRY(b, batch_launch_any(b, 0, 1));
    BHIP_TRY(b, hipEventRecord(ev.second, b->stream));
    b->timer.live.push_back(ev);
  }
  if (!b->member_streams.empty()) {
    BHIP_TRY(b, hipEventRecord(b->done_ev, b->stream));
    for (hipStream_t ms : b->member_streams) BHIP_TRY(b, hipStreamWaitEvent(ms, b->done_ev, 0));
  }
  return QMC_OK;
}

qmc_status qmc_batch_timing(qmc_batch b, double* total_ms, int64_t* sweeps, int32_t reset) {
  if (!b) return bfail(nullptr, QMC_ERR_ARG, "batch is NULL");
  BHIP_TRY(b, hipSetDevice(b->device));
  TimerClass& tc = b->timer;
  if (!tc.live.empty()) BHIP_TRY(b, hipEventSynchronize(tc.live.back().second));
  for (auto& ev : tc.live) {
    float ms = 0.f;
    BHIP_TRY(b, hipEventElapsedTime(&ms, ev.first, ev.second));
    tc.ms += ms;
    tc.launches += 1;
    tc.pool.push_back(ev);
  }
  tc.live.clear();
  if (total_ms) *total_ms = tc.ms;
  if (sweeps) *sweeps = tc.launches;
  if (reset) { tc.ms = 0.0; tc.launches = 0; }
  return QMC_OK;
}

qmc_status qmc_batch_destroy(qmc_batch b) {
  if (!b) return QMC_OK;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  for (hipGraphExec_t g : b->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  for (hipEvent_t e : b->member_ev)
    if (e) (void)hipEventDestroy(e);
  if (b->done_ev) (void)hipEventDestroy(b->done_ev);
  for (auto& ev : b->timer.live) { (void)hipEventDestroy(ev.first); (void)hipEventDestroy(ev.second); }
  for (auto& ev : b->timer.pool) { (void)hipEventDestroy(ev.first); (void)hipEventDestroy(ev.second); }
  if (b->d_sysdev) (void)hipFree(b->d_sysdev);
  if (b->d_maps) (void)hipFree(b->d_maps);
  delete b;
  return QMC_OK;
}

const char* qmc_last_error(qmc_system s) {
  if (s) return s->err.c_str();
  return g_last_error.c_str();
}

int32_t qmc_max_delay_rank(const qmc_system_desc* desc) {
  if (validate(desc) != QMC_OK) return 0;
  SysParams P;
  std::memset(&P, 0, sizeof P);
  P.n_up = desc->n_up;
  P.n_dn = desc->n_dn;
  P.N = desc->n_up + desc->n_dn;
  P.n_ions = desc->n_ions;
  for (int K = 64; K >= 4; K >>= 1)
    if (delayed_feasible(P, tsize_of(desc->precision), K)) return K;
  return 1;
}

size_t qmc_estimate_device_bytes(const qmc_system_desc* desc, int32_t n_walkers, int32_t gx, int32_t gy,
                                 int32_t gz) {
  if (!desc || n_walkers < 1 || gx < 4 || gy < 4 || gz < 4) return 0;
  if (desc->n_up < 1 || desc->n_dn < 0 || desc->n_up + desc->n_dn > 1024) return 0;
  if (desc->precision != QMC_FP64 && desc->precision != QMC_MIXED) return 0;
  const int n_orb = desc->n_up > desc->n_dn ? desc->n_up : desc->n_dn;
  const size_t table = align_up((size_t)gx * gy * gz * padded_stride(n_orb, desc->precision) * tsize_of(desc->precision));
  return system_bytes(desc) + table + walker_sizes(desc->n_up, desc->n_dn, desc->precision, n_walkers, n_orb, desc->move_kind).total();
}

}  // extern "C"
