// qmc_device.hpp -- parameter blocks and device helpers shared by the HIP
// kernels of the particle-by-particle VMC library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qmc.h"

namespace qmc {

constexpr int kBlock = 256;           // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kComp = 5;              // value, d/dx, d/dy, d/dz, Laplacian
constexpr double kPi = 3.14159265358979323846;

// The wave index of thread tid (64 lanes per wave).  Read from the first lane it is a scalar
// the compiler knows to be the same over the wave: branches on it stay scalar and values set
// under them live in scalar registers, which leaves vector registers to the arrays.
__device__ __forceinline__ int wave_of(int tid) { return __builtin_amdgcn_readfirstlane(tid >> 6); }

// Orders this wave's LDS writes before its later LDS reads (lanes read what other lanes of the
// same wave wrote).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Radial function of a Jastrow term (section "Jastrow factors").
struct Radial {
  int kind;          // QMC_J_NONE / PADE / BSPLINE
  int M;             // B-spline: number of free control points
  double a, b;       // Pade: u = a r / (1 + b r)
  double rc;         // B-spline cutoff
  double inv_delta;  // M / rc
  // B-spline control points p_0..p_M followed by zeros, so that the four
  // coefficients p_n..p_{n+3} of any interval n <= M-1 are addressable.
  double p[QMC_MAX_KNOTS + 4];
};

struct Jastrow {
  Radial same;   // electron pairs of equal spin
  Radial opp;    // electron pairs of opposite spin
  Radial ei;     // electron-ion
};

// Everything a kernel needs to know about a system, passed by value.
struct SysParams {
  int n_up, n_dn, N;      // electrons per spin, total
  int n_orb, S;           // orbitals; padded orbital stride of table and value rows
  int gx, gy, gz;         // spline grid
  int W;                  // walkers
  int n_ions;
  int bstride;            // elements of one walker's two inverses
  double L, sigma;
  double tie_guard;       // mixed precision: relative half-width of the FP64 re-decision band
  uint32_t key0, key1;    // Philox key (seed)
  const double* ions;     // [n_ions][4] = x, y, z, Z
  Jastrow jas;
  // three-body e-e-I term (j3_on): coefficients [2][mei+1][mei+1][mee+1] in the parameter
  // block itself, so that the loops' uniform indices read them as scalar loads; cutoff h
  int j3_on, j3_mei, j3_mee;
  double j3_h;
  double j3_g[2 * 4 * 4 * 4];
};

// Device buffers of the walkers.  T is the orbital/inverse precision.
template <typename T>
struct Walkers {
  double* pos;        // [W][N][3], wrapped into [0, L)
  double* prop;       // [W][N][4]: proposed x, y, z and the acceptance uniform
  T* vgl;             // [2][W][N][5][S]: value, gradient, Laplacian rows (two buffers)
  uint8_t* cur;       // [W][N]: which vgl buffer holds electron i's current row
  T* binv;            // [W][bstride]: B_up (n_up x n_up) then B_dn, B[l][k] = (A^-1)[l][k]
  double* logdet;     // [W][2]
  int* sign;          // [W][2]
  uint8_t* acc;       // [W][N]: accept flags of the last sweep
  uint32_t* nacc;     // [W]: accepted moves in the last launch
  int* status;        // [W]: nonzero = singular matrix at the last rebuild
  double* val64;      // [2][W][N][S]: FP64 orbital values (mixed precision only, else null)
  uint32_t* nguard;   // [W]: moves re-decided in FP64 (cumulative; mixed precision)
  uint32_t* sweep_ctr;  // index of the next sweep (device side, so captured sweeps replay correctly)
  T* xinv;            // [W][bstride]: FP64-refined copy of binv the measurement reads (mixed only, else null)
  int row_flip;       // rebuilds: 1 = invert the rows of the buffer that does not hold the current row
  const double* drift_v;  // [W][N][3] or null: drift velocities grad ln|Psi| at the current positions;
                          // the sweep's proposals then take the mean r + sigma^2 v
  int vstride;        // elements from one value row of vgl to the next (kComp * S; S for FP64 value rows)
  // Mixed precision, particle-by-particle moves (all null otherwise).  A walker whose FP32
  // inverse cannot carry FP64 decisions (an ill-conditioned Slater matrix) runs its chain in
  // FP64 on binv64 until its conditioning allows FP32 again.
  double* binv64;     // [W][bstride]: FP64 inverses; current for the walkers with fb[w] = 1
                      // (and, with drift moves, for every walker: the velocities read them)
  int* fb;            // [W]: 1 = FP64 fallback walker
  int fb_sel;         // chain launches advance only the walkers with fb[w] == fb_sel
  double* eta;        // [W][4]: ||I - A B||_F of each spin's inverse at the last check, then ||B||_F
  float* ecol;        // [W][N]: ||(I - A B)[:, k]||_2 of each electron's inverse column at the last check
  uint32_t* eta_age;  // [W]: sweeps since eta was measured
  uint32_t* pstat;    // [W][2]: early FP64 rebuilds, sweeps run in FP64 fallback (cumulative)
  const T* table;     // the orbital table (the measurement of fallback walkers evaluates it in FP64)
  // Mixed precision with drift moves (else null): the FP64 gradient rows the gather computed,
  // [2][W][N][3][S] beside vgl's buffers, so that drift velocities are FP64 quantities.
  double* grad64;
};

// Walkers a chain launch skips: those of the other precision class.
template <typename T>
__device__ __forceinline__ bool chain_skips(const Walkers<T>& Wk, int w) {
  return Wk.fb && Wk.fb[w] != Wk.fb_sel;
}

// Mixed-precision guard: a safety factor on the measured inverse error (it grows with the
// updates of a sweep), and the thresholds of the FP64 fallback.
constexpr double kEtaSafety = 2.0;
constexpr double kEtaRebuild = 2e-3;   // measured ||I - A B||_F above this: rebuild the inverse in FP64
constexpr double kEtaEnter = 2e-4;     // a fresh FP32 inverse this far off: FP64 fallback
constexpr double kEtaLeave = 5e-5;     // a fallback walker returns to FP32 below this

// Relative error bound on an FP32 ratio R = v . B[:, k] that the inverse's own error causes:
// with A B = I - E, R - R_exact = -(v^T A^-1) E e_k, so |dR| <= ||v^T B|| ||E[:, k]||_2 (1 + O(||E||)).
// The updates of a sweep mix the columns' errors (an accepted move at column p adds E[:, p] t_j / R_p
// to every column j), so a column's measured norm is floored at the columns' mean ||E||_F / sqrt(n);
// the factor kEtaSafety (1 + sweeps since the measurement) covers the growth over the sweep.  The
// band widening of a move is inverse_error_coef(...) * ||v^T B|| / |R|.  Read once per spin block
// (walker_eta) and once per electron (the column), never inside the sequential move loop.
template <typename T>
__device__ __forceinline__ double walker_eta(const Walkers<T>& Wk, int w, int sp, int n) {
  if (!Wk.eta) return 0.0;
  const double rn = 1.0 / sqrt((double)n);
  const double eta = fmax(Wk.eta[4 * w + sp] * rn, (double)n * rn * 5.9604644775390625e-08);
  const double age = Wk.eta_age ? (double)Wk.eta_age[w] : 0.0;
  return 2.0 * kEtaSafety * (1.0 + age) * eta;
}
// The coefficient for electron i (column of its spin block), N electrons; weta = walker_eta(...).
template <typename T>
__device__ __forceinline__ double inverse_error_coef(const Walkers<T>& Wk, int w, int i, int N, double weta) {
  if (!Wk.eta || !Wk.ecol) return weta;
  const double age = Wk.eta_age ? (double)Wk.eta_age[w] : 0.0;
  return fmax(weta, 2.0 * kEtaSafety * (1.0 + age) * (double)Wk.ecol[(size_t)w * N + i]);
}

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// SC'11).  Counter (electron, sweep, walker, purpose << 16 | sub), key = seed.
// ---------------------------------------------------------------------------
enum Purpose : uint32_t { kInit = 1, kPropose = 2, kAccept = 3, kBranch = 4 };

__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t y0 = hi1 ^ c1 ^ k0, y2 = hi0 ^ c3 ^ k1;
    c0 = y0; c1 = lo1; c2 = y2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Two doubles in [0,1) from the top 53 bits of each 64-bit half of a block.
__device__ __forceinline__ void uniform_pair(const SysParams& P, uint32_t purpose, uint32_t sub,
                                             uint32_t walker, uint32_t sweep, uint32_t elec,
                                             double& u0, double& u1) {
  uint32_t c0 = elec, c1 = sweep, c2 = walker, c3 = (purpose << 16) | sub;
  philox10(c0, c1, c2, c3, P.key0, P.key1);
  const uint64_t x0 = (uint64_t)c0 | ((uint64_t)c1 << 32);
  const uint64_t x1 = (uint64_t)c2 | ((uint64_t)c3 << 32);
  u0 = (double)(x0 >> 11) * 0x1.0p-53;
  u1 = (double)(x1 >> 11) * 0x1.0p-53;
}

// wrap_cell and axis_weights round every product and sum on its own (no fused multiply-adds):
// the kernels that inline them then agree bitwise whatever the surrounding code.
__device__ __forceinline__ double wrap_cell(double x, double L) {
#pragma clang fp contract(off)
  double y = x - L * floor(x / L);
  return (y >= L) ? 0.0 : y;
}

__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }
// The same with the reciprocal of L precomputed (no division).
__device__ __forceinline__ double min_image(double d, double L, double invL) { return d - L * rint(d * invL); }

// Uniform cubic B-spline basis on one axis: for t = i0 + f the knots
// i0-1 .. i0+2 carry weights w, first derivatives dw and second derivatives
// d2w (already scaled by knots per bohr h).
struct Axis {
  int idx[4];
  double w[4], dw[4], d2w[4];
};

__device__ __forceinline__ void axis_weights(double x, double L, int G, Axis& a) {
#pragma clang fp contract(off)
  const double h = (double)G / L;
  const double t = wrap_cell(x, L) * h;
  const double fl = floor(t);
  int i0 = (int)fl;
  const double f = t - fl;
  const double f2 = f * f, f3 = f2 * f, g = 1.0 - f;
  a.w[0] = g * g * g * (1.0 / 6.0);
  a.w[1] = (3.0 * f3 - 6.0 * f2 + 4.0) * (1.0 / 6.0);
  a.w[2] = (-3.0 * f3 + 3.0 * f2 + 3.0 * f + 1.0) * (1.0 / 6.0);
  a.w[3] = f3 * (1.0 / 6.0);
  a.dw[0] = -0.5 * g * g * h;
  a.dw[1] = (1.5 * f2 - 2.0 * f) * h;
  a.dw[2] = (-1.5 * f2 + f + 0.5) * h;
  a.dw[3] = 0.5 * f2 * h;
  const double h2 = h * h;
  a.d2w[0] = g * h2;
  a.d2w[1] = (3.0 * f - 2.0) * h2;
  a.d2w[2] = (1.0 - 3.0 * f) * h2;
  a.d2w[3] = f * h2;
  if (i0 >= G) i0 -= G;
  i0 = i0 < 0 ? 0 : (i0 > G - 1 ? G - 1 : i0);   // never index outside the table
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    int j = i0 - 1 + m;
    j = (j < 0) ? j + G : (j >= G ? j - G : j);
    a.idx[m] = j;
  }
}

// Radial Jastrow function value and first two derivatives.
// Cubic B-spline radial function on the knot interval holding t = r / delta: the four
// coefficients p[n..n+3] (n = floor t) give the interval's polynomial in f = t - n,
//   c0 = (p0 + 4 p1 + p2) / 6, c1 = (p2 - p0) / 2, c2 = (p0 - 2 p1 + p2) / 2,
//   c3 = (p3 - p0) / 6 + (p1 - p2) / 2,
// the expansion of the uniform cubic B-spline weights, evaluated by Horner's rule.
__device__ __forceinline__ void radial_eval(const Radial& R, double r, double& u, double& du,
                                            double& d2u) {
  if (R.kind == QMC_J_PADE) {
    const double d = 1.0 + R.b * r, id = 1.0 / d;
    u = R.a * r * id;
    du = R.a * id * id;
    d2u = -2.0 * R.a * R.b * id * id * id;
  } else if (R.kind == QMC_J_BSPLINE) {
    // branch-free in r: beyond the cutoff the first interval is evaluated and weighted zero
    const bool in = r < R.rc;
    const double t = in ? r * R.inv_delta : 0.0;
    const double fl = floor(t);
    const double* p = R.p + (int)fl;
    const double f = t - fl;
    const double p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3];
    const double c0 = (p0 + 4.0 * p1 + p2) * (1.0 / 6.0), c1 = 0.5 * (p2 - p0);
    const double c2 = 0.5 * (p0 + p2) - p1, c3 = (p3 - p0) * (1.0 / 6.0) + 0.5 * (p1 - p2);
    u = in ? c0 + f * (c1 + f * (c2 + f * c3)) : 0.0;
    du = in ? (c1 + f * (2.0 * c2 + 3.0 * f * c3)) * R.inv_delta : 0.0;
    d2u = in ? (2.0 * c2 + 6.0 * f * c3) * (R.inv_delta * R.inv_delta) : 0.0;
  } else {
    u = 0.0; du = 0.0; d2u = 0.0;
  }
}

__device__ __forceinline__ double radial_value(const Radial& R, double r) {
  if (R.kind == QMC_J_PADE) return R.a * r / (1.0 + R.b * r);
  if (R.kind == QMC_J_BSPLINE) {
    const bool in = r < R.rc;
    const double t = in ? r * R.inv_delta : 0.0;
    const double fl = floor(t);
    const double* p = R.p + (int)fl;
    const double f = t - fl;
    const double p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3];
    const double c0 = (p0 + 4.0 * p1 + p2) * (1.0 / 6.0), c1 = 0.5 * (p2 - p0);
    const double c2 = 0.5 * (p0 + p2) - p1, c3 = (p3 - p0) * (1.0 / 6.0) + 0.5 * (p1 - p2);
    return in ? c0 + f * (c1 + f * (c2 + f * c3)) : 0.0;
  }
  return 0.0;
}

// Three-body electron-electron-ion term for electrons i, j near one ion (section "Jastrow
// factors", the form of Drummond et al.): a = r_iI, b = r_jI, c = r_ij,
//   u = sum_{l,m,n} g_lmn a^l b^m c^n (a - h)^3 (b - h)^3, zero unless a < h and b < h.
// SAME selects the coefficient set (equal or opposite spins) at compile time, so that every
// coefficient index is uniform across the wave; u3_value / u3_derivs branch to it.
template <bool SAME>
__device__ __forceinline__ double u3_value_t(const SysParams& P, double a, double b, double c) {
  const double h = P.j3_h;
  if (a >= h || b >= h) return 0.0;
  const int M1 = P.j3_mei + 1, N1 = P.j3_mee + 1;
  const int g0 = SAME ? 0 : M1 * M1 * N1;
  double pa = 0.0;
  for (int l = M1 - 1; l >= 0; --l) {
    double pb = 0.0;
    for (int m = M1 - 1; m >= 0; --m) {
      const int gl = g0 + (l * M1 + m) * N1;
      double pc = 0.0;
      for (int n = N1 - 1; n >= 0; --n) pc = pc * c + P.j3_g[gl + n];
      pb = pb * b + pc;
    }
    pa = pa * a + pb;
  }
  const double fa = (a - h) * (a - h) * (a - h), fb = (b - h) * (b - h) * (b - h);
  return pa * fa * fb;
}

__device__ __forceinline__ double u3_value(const SysParams& P, bool same, double a, double b, double c) {
  return same ? u3_value_t<true>(P, a, b, c) : u3_value_t<false>(P, a, b, c);
}

// The same with its partial derivatives at fixed b: d = (u, u_a, u_c, u_aa, u_cc, u_ac).
template <bool SAME>
__device__ __forceinline__ void u3_derivs_t(const SysParams& P, double a, double b, double c, double d[6]) {
  const double h = P.j3_h;
  d[0] = d[1] = d[2] = d[3] = d[4] = d[5] = 0.0;
  if (a >= h || b >= h) return;
  const int M1 = P.j3_mei + 1, N1 = P.j3_mee + 1;
  const int g0 = SAME ? 0 : M1 * M1 * N1;
  double Pv = 0.0, Pa = 0.0, Pc = 0.0, Paa = 0.0, Pcc = 0.0, Pac = 0.0;
  double al = 1.0, al1 = 0.0, al2 = 0.0;   // a^l, l a^(l-1), l (l-1) a^(l-2) (likewise for c)
  for (int l = 0; l < M1; ++l) {
    double bm = 1.0;
    for (int m = 0; m < M1; ++m) {
      const int gl = g0 + (l * M1 + m) * N1;
      double cn = 1.0, cn1 = 0.0, cn2 = 0.0;
      for (int n = 0; n < N1; ++n) {
        const double gb = P.j3_g[gl + n] * bm;
        Pv += gb * al * cn;
        Pa += gb * al1 * cn;
        Paa += gb * al2 * cn;
        Pc += gb * al * cn1;
        Pcc += gb * al * cn2;
        Pac += gb * al1 * cn1;
        // next n: (n+1) n c^(n-1) = (n+1) cn1, (n+1) c^n = (n+1) cn, c^(n+1)
        cn2 = (n + 1) * cn1;
        cn1 = (n + 1) * cn;
        cn *= c;
      }
      bm *= b;
    }
    al2 = (l + 1) * al1;
    al1 = (l + 1) * al;
    al *= a;
  }
  const double t = a - h, fa = t * t * t, fa1 = 3.0 * t * t, fa2 = 6.0 * t;
  const double fb = (b - h) * (b - h) * (b - h);
  d[0] = Pv * fa * fb;
  d[1] = (Pa * fa + Pv * fa1) * fb;
  d[2] = Pc * fa * fb;
  d[3] = (Paa * fa + 2.0 * Pa * fa1 + Pv * fa2) * fb;
  d[4] = Pcc * fa * fb;
  d[5] = (Pac * fa + Pc * fa1) * fb;
}

__device__ __forceinline__ void u3_derivs(const SysParams& P, bool same, double a, double b, double c, double d[6]) {
  if (same) u3_derivs_t<true>(P, a, b, c, d);
  else u3_derivs_t<false>(P, a, b, c, d);
}

// Wave64 sum of a double (xor butterfly: every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One DPP step: v + (the value of the lane selected by ctrl), for the rows in
// row_mask (other rows add zero).  Works on the two 32-bit halves of a double.
template <int ctrl, int row_mask>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, ctrl, row_mask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, row_mask, 0xF, false);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave64 sum through the data-parallel-primitive lane network (no LDS round
// trips): pairs, quads, half rows and rows of 16, then the two row
// broadcasts carry the partial sums up to lane 63, read back as a uniform
// value.  All 64 lanes must be active.  The summation order is fixed.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xF>(v);   // row_half_mirror
  v = dpp_add<0x140, 0xF>(v);   // row_mirror
  v = dpp_add<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A value every lane of the wave holds alike, moved to scalar registers.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 16x16x4 matrix-core products.  Operands: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; result register r of lane l holds D[row(l, r)][l % 16],
// where the row mapping differs between the FP32 and FP64 instructions.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Workgroup barrier that orders LDS only: outstanding global loads (e.g. a
// prefetch) stay in flight across it.  Use __syncthreads() where global
// memory written by one wave is read by another.
__device__ __forceinline__ void sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace qmc
