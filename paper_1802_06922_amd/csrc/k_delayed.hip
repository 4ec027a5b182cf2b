// k_delayed.hip -- the move chain with rank-K delayed inverse updates.
//
// Section "Multi-Determinant Slater-Jastrow Form" names two ways of keeping
// the inverse current: single-row Sherman-Morrison updates and a delayed
// update that defers accepted row changes and applies them with
// matrix-matrix products (section "Performance and Parallel Scaling").  This
// kernel implements the delayed form in its Woodbury algebra, organised
// around the fact that every proposal row of a sweep is already known when
// the chain runs (the gather kernel evaluated them all).
//
// Window of K consecutive moves of one spin block, inverse B0 at its start,
// proposal rows v_q (q = 0..K-1, electron p = k0 + q):
//   Y = V B0                       (K x n: one matrix product per window)
// After m accepted moves (electrons P = p_1..p_m, window slots Q), with
//   C = Y[Q, P]   (m x m; the Woodbury capacitance I + Delta B0 E_P)
// the ratio of the next proposal (slot q, electron p) is the Schur complement
//   R = Y[q][p] - Y[q, P] C^-1 Y[Q, p]
// and acceptance borders C^-1 by one row and column.  At the window end the
// inverse becomes
//   B = B0 - B0[:, P] C^-1 (Y[Q, :] - E_P^T)      (rank-m product)
// which equals m successive Sherman-Morrison updates in exact arithmetic.
//
// The Jastrow change splits the same way: partners outside the window do not
// move during it, so their terms are summed for all K moves at once; only the
// K x K in-window terms depend on earlier decisions of the window, and both of
// their possible values are precomputed.
//
// Per window: a parallel phase (window rows, Jastrow sums, Y on the matrix
// cores), a sequential phase in one wave (O(m^2 + K) per move, no workgroup
// barriers), and the flush product on the matrix cores.
#include <cstdlib>

#include "qmc_guard.hpp"
#include "qmc_kernels.hpp"

namespace qmc {

constexpr int kMaxWindow = 64;
constexpr int kLdsIonsD = 256;

struct DLayout {
  size_t pos, prop, ions, red, jtab, rmag, tn, vpre, gold, gdiff, cur, acc, plist, qlist, vwin, ywin, zwin, gx, gr,
      grow, b, total;
};

// Intervals of a B-spline radial function's coefficient table: the M intervals below the cutoff
// and the one at it (a distance just below rc can round to t = M).
constexpr int kJTabInt = QMC_MAX_KNOTS + 1;

__host__ __device__ inline int round16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline DLayout dlayout(int N, int nmax, int n_ions, int ldl, size_t ts, bool b_in_lds,
                                           int K, bool prefetch = false) {
  DLayout L;
  const int nP = round16(nmax);
  size_t o = 0;
  auto al = [&](size_t a) { o = (o + a - 1) & ~(a - 1); };
  L.pos = o; o += sizeof(double) * 3 * N;
  L.prop = o; o += sizeof(double) * 4 * nmax;
  L.ions = o; o += (n_ions <= kLdsIonsD) ? sizeof(double) * 4 * n_ions : 0;
  L.red = o; o += sizeof(double) * kBlock;
  L.jtab = o; o += sizeof(double) * 3 * kJTabInt * 4;   // same-spin, opposite-spin, electron-ion
  L.rmag = o; o += (ts == 4) ? sizeof(double) * kBlock : 0;   // mixed: |v| . |B0[:, k]| partials
  L.tn = o; o += (ts == 4) ? sizeof(double) * kBlock : 0;     // mixed: |v^T B0|^2 partials
  al(16);
  L.vpre = o; o += prefetch ? ts * (size_t)K * (nP + 1) : 0;    // the next window's rows, prefetched
  // gold's storage later holds the window block yk with rows of K + 1 (bank spread) and
  // up to 7 entries read past its last row
  L.gold = o; o += sizeof(double) * ((size_t)K * (K + 1) + 8);
  L.gdiff = o; o += sizeof(double) * K * K;
  L.cur = o; o += nmax;
  L.acc = o; o += nmax;
  al(16);
  L.plist = o; o += sizeof(int) * K;
  L.qlist = o; o += sizeof(int) * K;
  al(16);
  // Window rows V (dead after Y = V B0) share storage with the flush's Z, and the
  // flush's U = B0[:, P] reuses Y's storage once Z has been formed.
  L.ywin = o; o += ts * (size_t)K * (nP + 1);   // Y rows (stride nP), or U transposed (stride nP + 1)
  al(16);
  L.zwin = o; o += ts * (size_t)K * (nP + 1);   // Z rows (stride nP), or the window rows (stride nP + 1)
  L.vwin = L.zwin;
  al(16);
  L.gx = o; o += (ts == 4) ? sizeof(double) * nP : 0;   // FP64 re-decision scratch (mixed)
  L.gr = o; o += (ts == 4) ? sizeof(double) * nP : 0;
  L.grow = o; o += (ts == 4) ? ts * (size_t)nP : 0;        // the re-decided move's row
  al(16);
  L.b = o; o += b_in_lds ? ts * (size_t)nmax * ldl : 0;
  L.total = o;
  return L;
}

template <bool BLDS>
__device__ __forceinline__ void dsync() {
  if (BLDS) sync_lds();
  else __syncthreads();
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The polynomial of B-spline interval i of R in f = t - i (the coefficients of radial_value),
// rounded one operation at a time.
__device__ __forceinline__ void bspline_interval(const Radial& R, int i, double* c) {
#pragma clang fp contract(off)
  const double* p = R.p + i;
  const double p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3];
  c[0] = (p0 + 4.0 * p1 + p2) * (1.0 / 6.0);
  c[1] = 0.5 * (p2 - p0);
  c[2] = 0.5 * (p0 + p2) - p1;
  c[3] = (p3 - p0) * (1.0 / 6.0) + 0.5 * (p1 - p2);
}

// u(r) of R with a B-spline's interval polynomials read from tab (kJTabInt x 4) instead of formed
// from the control points at every call.
__device__ __forceinline__ double radial_tab(const Radial& R, const double* tab, double r) {
  if (R.kind != QMC_J_BSPLINE) return radial_value(R, r);
  const bool in = r < R.rc;
  const double t = in ? r * R.inv_delta : 0.0;
  const double fl = floor(t);
  const double* c = tab + 4 * (int)fl;
  const double f = t - fl;
  return in ? fma(f, fma(f, fma(f, c[3], c[2]), c[1]), c[0]) : 0.0;
}

__device__ __forceinline__ double ju(const Jastrow& J, int kind, double r) {
  return kind == 0 ? radial_value(J.same, r) : (kind == 1 ? radial_value(J.opp, r) : radial_value(J.ei, r));
}

__device__ __forceinline__ double dist(double ax, double ay, double az, double bx, double by, double bz,
                                       double L, double invL) {
  double dx = ax - bx, dy = ay - by, dz = az - bz;
  dx -= L * rint(dx * invL);
  dy -= L * rint(dy * invL);
  dz -= L * rint(dz * invL);
  return sqrt(dx * dx + dy * dy + dz * dz);
}

// Matrix-core tiles of a wave are processed in groups of kGroup: their operand
// loads are issued together, so that when B lives in global memory a wave has
// several loads in flight instead of one round trip per 16 x 16 x 4 step.
// Four tiles for FP32; two for FP64, whose operands take twice the registers.
template <typename T> struct Group { static constexpr int n = sizeof(T) == 4 ? 4 : 2; };

// Y[q][c] = sum_l V[q][l] B[l][c] for q < Kw, c < n (all threads of the block).
template <typename T, bool MF>
__device__ __forceinline__ void gemm_window(const T* V, const T* B, int ldb, T* Y, int Kw, int n, int nP,
                                            int tid) {
  if (MF) {
    typedef Mfma<T> M;
    constexpr int kGroup = Group<T>::n;
    const int lane = tid & 63, wave = wave_of(tid), li = lane & 15, lk = lane >> 4;
    const int tq = (Kw + 15) >> 4, tc = (n + 15) >> 4, nt = tq * tc;
    // wave w takes tiles w, w + kWaves, ... in groups of kGroup
    for (int g0 = wave; g0 < nt; g0 += kWaves * kGroup) {
      typename M::v4 acc[kGroup];
      int qa[kGroup], cb[kGroup];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const int t = g0 + j * kWaves;
        acc[j] = typename M::v4{T(0), T(0), T(0), T(0)};
        qa[j] = t < nt ? (t / tc) * 16 + li : Kw;    // rows beyond Kw and columns beyond n read zero
        cb[j] = t < nt ? (t % tc) * 16 + li : n;
      }
#pragma unroll 2
      for (int l0 = 0; l0 < n; l0 += 4) {
        const int l = l0 + lk;
        T a[kGroup], b[kGroup];
        // unconditional loads from clamped indices (in bounds), out-of-range entries zeroed
        const int lc = l < n ? l : n - 1;
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
          const T av = V[(size_t)(qa[j] < Kw ? qa[j] : Kw - 1) * nP + lc];
          const T bv = B[(size_t)lc * ldb + (cb[j] < n ? cb[j] : n - 1)];
          a[j] = (qa[j] < Kw && l < n) ? av : T(0);
          b[j] = (l < n && cb[j] < n) ? bv : T(0);
        }
#pragma unroll
        for (int j = 0; j < kGroup; ++j) acc[j] = M::mma(a[j], b[j], acc[j]);
      }
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const int t = g0 + j * kWaves;
        if (t >= nt) continue;
        const int q0 = (t / tc) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q0 + M::row(lane, r);
          if (q < Kw && cb[j] < n) Y[(size_t)q * nP + cb[j]] = acc[j][r];
        }
      }
    }
  } else {
    for (int idx = tid; idx < Kw * n; idx += kBlock) {
      const int q = idx / n, c = idx - q * n;
      T acc = T(0);
      for (int l = 0; l < n; ++l) acc += V[(size_t)q * nP + l] * B[(size_t)l * ldb + c];
      Y[(size_t)q * nP + c] = acc;
    }
  }
}

// Z[r][c] = sum_l Cinv[r][l] (Y[q_l][c] - [c == p_l]) for r < mP, c < nz (rows from m and
// columns from n zero) on the FP64 matrix cores; wave w takes the 16 x 16 tiles w, w + kWaves,
// ...  Loads use clamped indices (always in bounds) and zero what lies outside.
template <typename T>
__device__ __forceinline__ void capacitance_z(const double* cinv, int K, const T* Y, int nP, const int* qlist,
                                              const int* plist, int m, int mP, int n, int nz, T* Z, int lane,
                                              int wave) {
  typedef Mfma<double> M;
  const int li = lane & 15, lk = lane >> 4;
  const int tr = (mP + 15) >> 4, tc = (nz + 15) >> 4;
  for (int t = wave; t < tr * tc; t += kWaves) {
    const int r0 = (t / tc) * 16, r = r0 + li, c = (t % tc) * 16 + li;
    const int rc = r < m ? r : m - 1, cc = c < n ? c : n - 1;
    typename M::v4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < m; l0 += 4) {
      const int l = l0 + lk, lc = l < m ? l : m - 1;
      const double av = cinv[rc * K + lc];
      const double yv = (double)Y[(size_t)qlist[lc] * nP + cc] - (cc == plist[lc] ? 1.0 : 0.0);
      acc = M::mma((r < m && l < m) ? av : 0.0, (l < m && c < n) ? yv : 0.0, acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = r0 + M::row(lane, q);
      if (rr < mP && c < nz) Z[(size_t)rr * nP + c] = (T)acc[q];
    }
  }
}

// B[l][c] -= sum_r U[l][r] Z[r][c] for l, c < n, r < mP (U, Z zero-padded to mP).
template <typename T, bool MF>
__device__ __forceinline__ void gemm_flush(T* B, int ldb, const T* U, int ldu, const T* Z, int nP, int n,
                                           int mP, int tid) {
  if (MF) {
    typedef Mfma<T> M;
    constexpr int kGroup = Group<T>::n;
    const int lane = tid & 63, wave = wave_of(tid), li = lane & 15, lk = lane >> 4;
    const int tt = (n + 15) >> 4, nt = tt * tt;
    for (int g0 = wave; g0 < nt; g0 += kWaves * kGroup) {
      // the old values of the group's tiles are loaded first; they arrive while the products run
      T old[kGroup][4];
      int lrow[kGroup], cb[kGroup];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const int t = g0 + j * kWaves;
        lrow[j] = t < nt ? (t / tt) * 16 : n;
        cb[j] = t < nt ? (t % tt) * 16 + li : n;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = lrow[j] + M::row(lane, r);
          const T v = B[(size_t)(l < n ? l : n - 1) * ldb + (cb[j] < n ? cb[j] : n - 1)];
          old[j][r] = (l < n && cb[j] < n) ? v : T(0);
        }
      }
      typename M::v4 acc[kGroup];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) acc[j] = typename M::v4{T(0), T(0), T(0), T(0)};
      for (int r0 = 0; r0 < mP; r0 += 4) {
        const int r = r0 + lk;
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
          const int la = lrow[j] + li;
          const T av = U[(size_t)(la < n ? la : n - 1) * ldu + r];
          const T bv = Z[(size_t)r * nP + (cb[j] < n ? cb[j] : n - 1)];
          acc[j] = M::mma(la < n ? av : T(0), cb[j] < n ? bv : T(0), acc[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < kGroup; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = lrow[j] + M::row(lane, r);
          if (l < n && cb[j] < n) B[(size_t)l * ldb + cb[j]] = old[j][r] - acc[j][r];
        }
    }
  } else {
    for (int idx = tid; idx < n * n; idx += kBlock) {
      const int l = idx / n, c = idx - l * n;
      T acc = T(0);
      for (int r = 0; r < mP; ++r) acc += U[(size_t)l * ldu + r] * Z[(size_t)r * nP + c];
      B[(size_t)l * ldb + c] -= acc;
    }
  }
}

// The flush for an inverse in global memory.  There the product is bound by the latency
// of the B loads, not by arithmetic: each thread updates blocks of 4 rows by 16 bytes of
// columns (4 FP32 or 2 FP64) with 16-byte loads and stores, kFlushBatch blocks at a
// time, so a wave keeps 4 kFlushBatch wide loads in flight; consecutive threads take
// consecutive column blocks of the same rows (coalesced).  Needs n a multiple of 4, ldb a
// multiple of the vector width, and B, Z 16-byte aligned.
constexpr int kFlushBatch = 2;
template <typename T>
__device__ __forceinline__ void flush_global(T* B, int ldb, const T* U, int ldu, const T* Z, int nP, int n,
                                             int mP, int tid) {
  constexpr int V = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(V)));
  const int cbn = n / V, nb = (n >> 2) * cbn;
  for (int b0 = tid; b0 < nb; b0 += kBlock * kFlushBatch) {
    vec old[kFlushBatch][4], acc[kFlushBatch][4];
    int lr[kFlushBatch], cv[kFlushBatch];
#pragma unroll
    for (int j = 0; j < kFlushBatch; ++j) {
      const int b = min(b0 + j * kBlock, nb - 1);   // clamped: loads stay in bounds
      lr[j] = (b / cbn) * 4;
      cv[j] = (b - (b / cbn) * cbn) * V;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        old[j][i] = *reinterpret_cast<const vec*>(B + (size_t)(lr[j] + i) * ldb + cv[j]);
        acc[j][i] = vec(T(0));
      }
    }
#pragma unroll 1
    for (int r = 0; r < mP; ++r) {
#pragma unroll
      for (int j = 0; j < kFlushBatch; ++j) {
        const vec z = *reinterpret_cast<const vec*>(Z + (size_t)r * nP + cv[j]);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[j][i] += U[(size_t)(lr[j] + i) * ldu + r] * z;
      }
    }
#pragma unroll
    for (int j = 0; j < kFlushBatch; ++j) {
      if (b0 + j * kBlock >= nb) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        *reinterpret_cast<vec*>(B + (size_t)(lr[j] + i) * ldb + cv[j]) = old[j][i] - acc[j][i];
    }
  }
}

// ---------------------------------------------------------------------------
// The active spin block's inverse in registers for the whole sweep (FP32, spin blocks of up to
// 16 NT electrons; used where the inverse does not fit the LDS).  B is cut into 16 x 16 tiles;
// wave v owns the column tiles v, v + kWaves, ..., each with all its row tiles, in the layout
// of a matrix-core accumulator: register r of tile (rt, ct) in lane l holds
// B[16 rt + 4 (l / 16) + r][16 ct + l % 16].  Register r of a tile is also the second operand
// of one 16x16x4 product step whose k index g = l / 16 stands for row 16 rt + 4 g + r, so the
// window product Y = V B0 runs on the matrix cores straight from the registers (the first
// operand, V, is read from LDS with the same row order), and the flush's rank-m update
// accumulates into the tiles in place.  The inverse is read from and written to HBM once per
// spin block and sweep.  Padding rows and columns (>= n) hold zeros throughout.
// ---------------------------------------------------------------------------
template <int NT> struct RegTiles {
  static constexpr int CT = (NT + kWaves - 1) / kWaves;
  typedef float v4 __attribute__((ext_vector_type(4)));
  v4 t[CT][NT];
};
template <> struct RegTiles<0> { static constexpr int CT = 0; };

// An LDS offset the compiler must take as computed here: addresses derived from it fold into
// the instructions' immediate offsets at the point of use instead of being precomputed once for
// every tile and kept live across the sweep (which spills the tiles).
__device__ __forceinline__ int pinned(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// This lane's index, computed afresh at each call: an address derived from it is then formed
// where it is used instead of being kept live (and spilled) across the sweep.
__device__ __forceinline__ int lane_now() {
  int l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
  return l;
}

// HBM <-> tiles through an LDS slab of 16 rows (stage: 16 n floats): the 16 rows of a row tile
// are one contiguous stretch of B, read or written by the whole workgroup, and each lane moves
// its entries between the slab and its registers.  All threads call these.
template <int NT>
__device__ __forceinline__ void regb_load(RegTiles<NT>& R, const float* __restrict__ Bg, float* stage, int n, int nt,
                                          int lane, int wave, int tid) {
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < NT; ++rt) {
    if (rt < nt) {
      const int rows = min(16, n - 16 * rt);
      const float* src = Bg + (size_t)16 * rt * n;
      for (int q = tid; q < rows * n; q += kBlock) stage[q] = src[q];
      __syncthreads();
#pragma unroll
      for (int cj = 0; cj < RegTiles<NT>::CT; ++cj) {
        const int ct = wave + kWaves * cj, c = 16 * ct + i;
        const int base = pinned(4 * g * n + (c < n ? c : 0));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = 4 * g + r;
          const float v = stage[l < rows ? base + r * n : 0];
          R.t[cj][rt][r] = (ct < nt && l < rows && c < n) ? v : 0.0f;
        }
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int cj = 0; cj < RegTiles<NT>::CT; ++cj)
#pragma unroll
        for (int r = 0; r < 4; ++r) R.t[cj][rt][r] = 0.0f;
    }
  }
}

template <int NT>
__device__ __forceinline__ void regb_store(const RegTiles<NT>& R, float* __restrict__ Bg, float* stage, int n,
                                           int nt, int lane, int wave, int tid) {
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < NT; ++rt) {
    if (rt < nt) {
      const int rows = min(16, n - 16 * rt);
#pragma unroll
      for (int cj = 0; cj < RegTiles<NT>::CT; ++cj) {
        const int ct = wave + kWaves * cj, c = 16 * ct + i;
        const int base = pinned(4 * g * n + c);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = 4 * g + r;
          if (ct < nt && l < rows && c < n) stage[base + r * n] = R.t[cj][rt][r];
        }
      }
      __syncthreads();
      float* dst = Bg + (size_t)16 * rt * n;
      for (int q = tid; q < rows * n; q += kBlock) dst[q] = stage[q];
      __syncthreads();
    }
  }
}

// Y[q][c] = sum_l V[q][l] B0[l][c] for q < Kw <= 32 and the columns of this wave's tiles (V: LDS,
// row stride ldv, columns up to 16 nt zero past n; Y: LDS, row stride nP).
template <int NT>
__device__ __forceinline__ void regb_window(const RegTiles<NT>& R, const float* V, int ldv, float* Y, int nP, int Kw,
                                            int nt, int lane, int wave) {
  typedef typename RegTiles<NT>::v4 v4;
  constexpr int CT = RegTiles<NT>::CT;
  const int i = lane & 15, g = lane >> 4;
  const bool two = Kw > 16;   // a second 16-row block of window rows
  // rows past the window (their products are discarded) read the window's last row: the window
  // buffer holds only Kw <= K rows
  const int v0 = pinned(min(i, Kw - 1) * ldv + 4 * g), v1 = pinned(min(16 + i, Kw - 1) * ldv + 4 * g);
  v4 acc[2][CT];
#pragma unroll
  for (int cj = 0; cj < CT; ++cj) {
    acc[0][cj] = v4{0.0f, 0.0f, 0.0f, 0.0f};
    acc[1][cj] = v4{0.0f, 0.0f, 0.0f, 0.0f};
  }
#pragma unroll
  for (int rt = 0; rt < NT; ++rt) {
    if (rt < nt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float a0 = V[v0 + 16 * rt + r];
        const float a1 = two ? V[v1 + 16 * rt + r] : 0.0f;
#pragma unroll
        for (int cj = 0; cj < CT; ++cj) {
          acc[0][cj] = Mfma<float>::mma(a0, R.t[cj][rt][r], acc[0][cj]);
          if (two) acc[1][cj] = Mfma<float>::mma(a1, R.t[cj][rt][r], acc[1][cj]);
        }
      }
    }
  }
  const int y0 = pinned(4 * g * nP + i);
#pragma unroll
  for (int cj = 0; cj < CT; ++cj) {
    const int ct = wave + kWaves * cj;
    if (ct >= nt) continue;
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 16 * qb + 4 * g + r;
        if (q < Kw) Y[y0 + (16 * qb + r) * nP + 16 * ct] = acc[qb][cj][r];
      }
  }
}

// mag[q] = sum_l |V[q][l]| |B0[l][k0 + q]| for the window columns this wave holds (the bound on the
// FP32 rounding of the window's ratios).  The four lanes holding a column add their rows.
template <int NT>
__device__ __forceinline__ void regb_magnitudes(const RegTiles<NT>& R, const float* V, int ldv, double* mag, int k0,
                                                int Kw, int n, int nt, int lane, int wave) {
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int cj = 0; cj < RegTiles<NT>::CT; ++cj) {
    const int ct = wave + kWaves * cj, c = 16 * ct + i, q = c - k0;
    const bool in = ct < nt && c < n && q >= 0 && q < Kw;
    double part = 0.0;
    if (in) {
      const int vb = pinned(q * ldv + 4 * g);
#pragma unroll
      for (int rt = 0; rt < NT; ++rt)
        if (rt < nt)
#pragma unroll
          for (int r = 0; r < 4; ++r) part += fabs((double)V[vb + 16 * rt + r]) * fabs((double)R.t[cj][rt][r]);
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (in && g == 0) mag[q] = part;
  }
}

// Ut[r][l] = B0[l][p_r] (r < m, l < 16 nt; rows m .. mP - 1 zero): U transposed, row stride ldt.
template <int NT>
__device__ __forceinline__ void regb_columns(const RegTiles<NT>& R, float* Ut, int ldt, const int* plist, int m,
                                             int mP, int nt, int lane, int wave, int tid) {
  const int i = lane & 15, g = lane >> 4, nc = 16 * nt;
  for (int idx = tid; idx < (mP - m) * nc; idx += kBlock) {
    const int r = m + idx / nc, l = idx % nc;
    Ut[(size_t)r * ldt + l] = 0.0f;
  }
  for (int r = 0; r < m; ++r) {
    const int p = plist[r], ct = p >> 4;
    if (ct % kWaves != wave || (p & 15) != i) continue;
    const int ub = pinned(r * ldt + 4 * g);
#pragma unroll
    for (int cj = 0; cj < RegTiles<NT>::CT; ++cj) {
      if (cj != ct / kWaves) continue;
#pragma unroll
      for (int rt = 0; rt < NT; ++rt)
        if (rt < nt)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) Ut[ub + 16 * rt + rr] = R.t[cj][rt][rr];
    }
  }
}

// B -= U Z in place in the tiles: Ut (LDS, U transposed, mP x 16 nt, stride ldt), Z (LDS,
// mP x 16 nt, stride nP, zero past column n).
template <int NT>
__device__ __forceinline__ void regb_flush(RegTiles<NT>& R, const float* Ut, int ldt, const float* Z, int nP, int mP,
                                           int nt, int lane, int wave) {
  constexpr int CT = RegTiles<NT>::CT;
  const int i = lane & 15, g = lane >> 4;
  for (int r0 = 0; r0 < mP; r0 += 4) {
    const int zb = pinned((r0 + g) * nP + i), ub = pinned((r0 + g) * ldt + i);
    float zf[CT];
#pragma unroll
    for (int cj = 0; cj < CT; ++cj) {
      const int ct = wave + kWaves * cj;
      const float z = Z[zb + 16 * (ct < nt ? ct : 0)];
      zf[cj] = ct < nt ? z : 0.0f;   // tiles past the matrix stay zero
    }
#pragma unroll
    for (int rt = 0; rt < NT; ++rt) {
      if (rt < nt) {
        const float a = -Ut[ub + 16 * rt];
#pragma unroll
        for (int cj = 0; cj < CT; ++cj) R.t[cj][rt] = Mfma<float>::mma(a, zf[cj], R.t[cj][rt]);
      }
    }
  }
}

// out[c] = (add ? out[c] : 0) + sum_l x[l] B[l][c] for the columns c < n of this wave's tiles,
// summed in FP64 from the FP32 tiles (x: LDS, zero from n up to 16 nt); the four lanes holding a
// column add their rows.
template <int NT, typename X>
__device__ __forceinline__ void regb_rowvec(const RegTiles<NT>& R, const X* x, double* out, bool add, int n, int nt,
                                            int lane, int wave) {
  const int i = lane & 15, g = lane >> 4;
  const int xb = pinned(4 * g);
#pragma unroll
  for (int cj = 0; cj < RegTiles<NT>::CT; ++cj) {
    const int ct = wave + kWaves * cj, c = 16 * ct + i;
    double part = 0.0;
    if (ct < nt) {
#pragma unroll
      for (int rt = 0; rt < NT; ++rt)
        if (rt < nt)
#pragma unroll
          for (int r = 0; r < 4; ++r) part += (double)x[xb + 16 * rt + r] * (double)R.t[cj][rt][r];
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (g == 0 && ct < nt && c < n) out[c] = add ? out[c] + part : part;
  }
}

// col[l] = B[l][k] for l < 16 nt (written by the four lanes that hold column k).
template <int NT>
__device__ __forceinline__ void regb_column(const RegTiles<NT>& R, float* col, int k, int nt, int lane, int wave) {
  const int i = lane & 15, g = lane >> 4, ct = k >> 4;
  if (ct % kWaves != wave || (k & 15) != i) return;
  const int cb = pinned(4 * g);
#pragma unroll
  for (int cj = 0; cj < RegTiles<NT>::CT; ++cj) {
    if (cj != ct / kWaves) continue;
#pragma unroll
    for (int rt = 0; rt < NT; ++rt)
      if (rt < nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) col[cb + 16 * rt + r] = R.t[cj][rt][r];
  }
}

// Sherman-Morrison in the tiles: B[l][c] -= col[l] (t[c] - delta_ck) / R for the accepted row of
// electron k (col = B[:, k], t = v^T B, R = t[k]; LDS).
template <int NT>
__device__ __forceinline__ void regb_rank1(RegTiles<NT>& R, const float* col, const float* t, float invR, int k,
                                           int n, int nt, int lane, int wave) {
  const int i = lane & 15, g = lane >> 4;
  const int cb = pinned(4 * g);
#pragma unroll
  for (int cj = 0; cj < RegTiles<NT>::CT; ++cj) {
    const int ct = wave + kWaves * cj, c = 16 * ct + i;
    if (ct >= nt) continue;
    const float f = c < n ? invR * (t[c] - (c == k ? 1.0f : 0.0f)) : 0.0f;
#pragma unroll
    for (int rt = 0; rt < NT; ++rt)
      if (rt < nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) R.t[cj][rt][r] -= col[cb + 16 * rt + r] * f;
  }
}

template <typename T, bool BLDS, bool MF, int RT>
__device__ __forceinline__ void chain_delayed_walker(const SysParams& P, const Walkers<T>& Wk, int w, int K,
                                                     int ldl) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Jastrow sj;
  __shared__ int sm_m, sm_stop;
  __shared__ double sm_dj;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_of(tid);
  if (chain_skips(Wk, w)) return;
  const int N = P.N, nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn, nP = round16(nmax);
  const DLayout lay = dlayout(N, nmax, P.n_ions, ldl, sizeof(T), BLDS, K, RT > 0);
  double* spos = reinterpret_cast<double*>(smem + lay.pos);
  double* sprop = reinterpret_cast<double*>(smem + lay.prop);
  const bool ions_lds = P.n_ions <= kLdsIonsD;
  double* sion = reinterpret_cast<double*>(smem + lay.ions);
  const double* ions = ions_lds ? sion : P.ions;
  double* red = reinterpret_cast<double*>(smem + lay.red);
  double* rmag = reinterpret_cast<double*>(smem + lay.rmag);
  double* tnp = reinterpret_cast<double*>(smem + lay.tn);
  double* gold = reinterpret_cast<double*>(smem + lay.gold);
  double* gdiff = reinterpret_cast<double*>(smem + lay.gdiff);
  uint8_t* scur = smem + lay.cur;
  uint8_t* sacc = smem + lay.acc;
  int* plist = reinterpret_cast<int*>(smem + lay.plist);
  int* qlist = reinterpret_cast<int*>(smem + lay.qlist);
  // (B): the window block, in FP64 (also in mixed precision: the K x K elimination and the
  // capacitance inverse are small, and FP32 rounding there compounds over the window)
  double* yk = reinterpret_cast<double*>(smem + lay.gold);
  T* vwin = reinterpret_cast<T*>(smem + lay.vwin);
  T* ywin = reinterpret_cast<T*>(smem + lay.ywin);
  T* ubuf = ywin;
  T* zwin = reinterpret_cast<T*>(smem + lay.zwin);
  double* sgx = reinterpret_cast<double*>(smem + lay.gx);
  double* sgr = reinterpret_cast<double*>(smem + lay.gr);
  T* sgrow = reinterpret_cast<T*>(smem + lay.grow);
  T* sB = reinterpret_cast<T*>(smem + lay.b);
  const double L = P.L, invL = 1.0 / P.L;
  const int tpq = kBlock / K;   // threads per window slot in the Jastrow sums
  // RT > 0: the active spin block's inverse lives in registers (breg) for the sweep; the window
  // rows are then stored with row stride nP + 1 (the product reads them across rows)
  RegTiles<RT> breg;
  const int ldv = RT > 0 ? nP + 1 : nP;
  T* vpre = reinterpret_cast<T*>(smem + lay.vpre);
  // rows of a window into dst: kA1 loads per thread in flight before their stores (the rows do not
  // depend on the chain, only the HBM latency matters); indices are clamped so every load is in
  // bounds; register mode zeroes the columns past n up to the tiles' 16 nt
  auto load_rows = [&](T* dst, size_t item0_, int kstart, int kw, int nt_, int n_, const uint8_t* cur_, int t0,
                       int tstride) {
    constexpr int kA1 = 8;
    const int nc = RT > 0 ? 16 * nt_ : n_, total = kw * nc;
    for (int b0 = t0; b0 < total; b0 += tstride * kA1) {
      T v[kA1];
#pragma unroll
      for (int e = 0; e < kA1; ++e) {
        const int idx = b0 + e * tstride;
        const bool ok = idx < total;
        const int q = ok ? idx / nc : 0, l = ok ? idx - q * nc : 0;
        const T x = Wk.vgl[((size_t)(1 - cur_[kstart + q]) * P.W * N + item0_ + kstart + q) * Wk.vstride +
                           (l < n_ ? l : 0)];
        v[e] = (ok && l < n_) ? x : T(0);
      }
#pragma unroll
      for (int e = 0; e < kA1; ++e) {
        const int idx = b0 + e * tstride;
        if (idx < total) {
          const int q = idx / nc, l = idx - q * nc;
          dst[(size_t)q * ldv + l] = v[e];
        }
      }
    }
  };
  const int ldy = K + 1;        // row stride of yk: the lanes' rows start in different banks
  // the wave that runs the moves in sequence rotates with the workgroup index, so that the
  // sequential phases of workgroups sharing a compute unit fall on different SIMDs
  const int seq_wave = (int)(blockIdx.x & (kWaves - 1)), seq_tid = seq_wave * 64;

  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.jas);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&sj);
    for (int q = tid; q < (int)(sizeof(Jastrow) / 4); q += kBlock) dst[q] = src[q];
  }
  // the radial functions' interval polynomials (read after the barriers before the first window)
  double* jtab = reinterpret_cast<double*>(smem + lay.jtab);
  for (int t = tid; t < 3 * kJTabInt; t += kBlock)
    bspline_interval(t < kJTabInt ? P.jas.same : (t < 2 * kJTabInt ? P.jas.opp : P.jas.ei), t % kJTabInt,
                     jtab + 4 * t);
  for (int j = tid; j < 3 * N; j += kBlock) spos[j] = Wk.pos[(size_t)w * 3 * N + j];
  if (ions_lds)
    for (int j = tid; j < 4 * P.n_ions; j += kBlock) sion[j] = P.ions[j];
  uint32_t nacc = 0, nguard = 0;

  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp ? P.n_dn : P.n_up;
    const int off = sp ? P.n_up : 0;
    if (n == 0) continue;
    const size_t item0 = (size_t)w * N + off;
    double logd = Wk.logdet[2 * w + sp];
    int sgn = Wk.sign[2 * w + sp];
    for (int q = tid; q < 4 * n; q += kBlock) sprop[q] = Wk.prop[item0 * 4 + q];
    for (int q = tid; q < n; q += kBlock) scur[q] = Wk.cur[item0 + q];
    T* Bg = Wk.binv + (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
    T* Bm;
    int ldb;
    if (BLDS) {
      for (int q = tid; q < n * n; q += kBlock) {
        const int l = q / n;
        sB[l * ldl + (q - l * n)] = Bg[q];
      }
      Bm = sB;
      ldb = ldl;
    } else {
      Bm = Bg;
      ldb = n;
    }
    const bool up_block = sp == 0;
    const int nt = (n + 15) >> 4;
    const double weta = sizeof(T) == 4 ? walker_eta(Wk, w, sp, n) : 0.0;   // mixed: inverse error of B
    if constexpr (RT > 0) regb_load<RT>(breg, Bg, reinterpret_cast<float*>(ywin), n, nt, lane, wave, tid);
    __syncthreads();   // the block's proposals, buffer flags and inverse are staged before any use

    int pre_k0 = -1;   // register mode: the window start whose rows vpre holds
    for (int k0 = 0; k0 < n;) {
      const int Kw = (n - k0) < K ? (n - k0) : K;
      // mixed: lane q's inverse-error coefficient of its electron's column (loaded here, used in
      // the sequential phase)
      const double ecq = (sizeof(T) == 4 && lane < Kw) ? inverse_error_coef(Wk, w, off + k0 + lane, N, weta) : 0.0;
      // (A1) the window's proposal rows, unless the previous window's moves prefetched them
      T* vcur = vwin;
      if (RT > 0 && pre_k0 == k0) {
        vcur = vpre;
      } else {
        load_rows(vwin, item0, k0, Kw, nt, n, scur, tid, kBlock);
        __syncthreads();
      }
      // (A2) Jastrow: fixed partners (outside the window) per slot, and in-window pair terms
      {
        const int q = tid / tpq, s = tid - q * tpq;
        double part = 0.0;
        if (q < Kw) {
          const int kq = k0 + q, iq = off + kq;
          const double px = sprop[4 * kq], py = sprop[4 * kq + 1], pz = sprop[4 * kq + 2];
          const double ox = spos[3 * iq], oy = spos[3 * iq + 1], oz = spos[3 * iq + 2];
          // partner ranges with one radial function each (no divergence between lanes):
          // same-spin electrons before and after the window, the other spin block, the ions
          auto range = [&](const Radial& R, const double* tab, int lo, int hi, const double* c, int stride) {
            for (int j = lo + s; j < hi; j += tpq) {
              const double* cj = c + (size_t)stride * j;
              part += radial_tab(R, tab, dist(px, py, pz, cj[0], cj[1], cj[2], L, invL)) -
                      radial_tab(R, tab, dist(ox, oy, oz, cj[0], cj[1], cj[2], L, invL));
            }
          };
          const int ooff = up_block ? P.n_up : 0, no = up_block ? P.n_dn : P.n_up;
          range(sj.same, jtab, off, off + k0, spos, 3);
          range(sj.same, jtab, off + k0 + Kw, off + n, spos, 3);
          range(sj.opp, jtab + 4 * kJTabInt, ooff, ooff + no, spos, 3);
          range(sj.ei, jtab + 8 * kJTabInt, 0, P.n_ions, ions, 4);
          if (P.j3_on) {
            // three-body terms with partners outside the window (in-window partners are pair
            // terms below), over the ions within the cutoff of r or r'
            const double h = P.j3_h;
            const int w0 = off + k0, w1 = off + k0 + Kw;
            // ions near r' or r, ascending; with at most 64 ions a lane visits only its own
            uint64_t near = 0;
            const bool masked = P.n_ions <= 64;
            if (masked)
              for (int I = 0; I < P.n_ions; ++I) {
                const double* ion = ions + 4 * I;
                if (dist(px, py, pz, ion[0], ion[1], ion[2], L, invL) < h ||
                    dist(ox, oy, oz, ion[0], ion[1], ion[2], L, invL) < h)
                  near |= 1ull << I;
              }
            for (int I = masked ? (near ? __builtin_ctzll(near) : P.n_ions) : 0; I < P.n_ions;
                 I = masked ? ((near &= near - 1) ? __builtin_ctzll(near) : P.n_ions) : I + 1) {
              const double* ion = ions + 4 * I;
              const double a1 = dist(px, py, pz, ion[0], ion[1], ion[2], L, invL);
              const double a0 = dist(ox, oy, oz, ion[0], ion[1], ion[2], L, invL);
              if (a1 >= h && a0 >= h) continue;
              for (int j = s; j < N; j += tpq) {
                if (j >= w0 && j < w1) continue;
                const double* cj = spos + 3 * j;
                const double b = dist(cj[0], cj[1], cj[2], ion[0], ion[1], ion[2], L, invL);
                if (b >= h) continue;
                const bool same = (j < P.n_up) == up_block;
                if (a1 < h) part += u3_value(P, same, a1, b, dist(px, py, pz, cj[0], cj[1], cj[2], L, invL));
                if (a0 < h) part -= u3_value(P, same, a0, b, dist(ox, oy, oz, cj[0], cj[1], cj[2], L, invL));
              }
            }
          }
        }
        red[tid] = part;
        if (sizeof(T) == 4 && RT == 0) {
          // magnitude of the ratio's terms, sum_l |v_l| |B0[l][k]|, which bounds the FP32
          // rounding of the ratio (mixed precision guard band)
          double mag = 0.0;
          if (q < Kw)
            for (int l = s; l < n; l += tpq)
              mag += fabs((double)vwin[(size_t)q * ldv + l]) * fabs((double)Bm[(size_t)l * ldb + k0 + q]);
          rmag[tid] = mag;
        }
      }
      for (int idx = tid; idx < Kw * Kw; idx += kBlock) {
        const int q = idx / Kw, q2 = idx - q * Kw;
        if (q == q2) continue;
        const int kq = k0 + q, k2 = k0 + q2, iq = off + kq, i2 = off + k2;
        const double px = sprop[4 * kq], py = sprop[4 * kq + 1], pz = sprop[4 * kq + 2];
        const double ox = spos[3 * iq], oy = spos[3 * iq + 1], oz = spos[3 * iq + 2];
        const double cx = spos[3 * i2], cy = spos[3 * i2 + 1], cz = spos[3 * i2 + 2];
        double g_old = ju(sj, 0, dist(px, py, pz, cx, cy, cz, L, invL)) -
                       ju(sj, 0, dist(ox, oy, oz, cx, cy, cz, L, invL));
        const double nx = sprop[4 * k2], ny = sprop[4 * k2 + 1], nz = sprop[4 * k2 + 2];
        double g_new = 0.0;
        if (q2 < q)
          g_new = ju(sj, 0, dist(px, py, pz, nx, ny, nz, L, invL)) -
                  ju(sj, 0, dist(ox, oy, oz, nx, ny, nz, L, invL));
        if (P.j3_on) {
          // three-body terms of the pair (same spin) over the ions near either electron
          const double h = P.j3_h;
          for (int I = 0; I < P.n_ions; ++I) {
            const double* ion = ions + 4 * I;
            const double a1 = dist(px, py, pz, ion[0], ion[1], ion[2], L, invL);
            const double a0 = dist(ox, oy, oz, ion[0], ion[1], ion[2], L, invL);
            if (a1 >= h && a0 >= h) continue;
            const double bo = dist(cx, cy, cz, ion[0], ion[1], ion[2], L, invL);
            if (bo < h) {
              if (a1 < h) g_old += u3_value(P, true, a1, bo, dist(px, py, pz, cx, cy, cz, L, invL));
              if (a0 < h) g_old -= u3_value(P, true, a0, bo, dist(ox, oy, oz, cx, cy, cz, L, invL));
            }
            if (q2 < q) {
              const double bn = dist(nx, ny, nz, ion[0], ion[1], ion[2], L, invL);
              if (bn < h) {
                if (a1 < h) g_new += u3_value(P, true, a1, bn, dist(px, py, pz, nx, ny, nz, L, invL));
                if (a0 < h) g_new -= u3_value(P, true, a0, bn, dist(ox, oy, oz, nx, ny, nz, L, invL));
              }
            }
          }
        }
        gold[q2 * K + q] = g_old;   // transposed: lane q reads column q
        if (q2 < q) gdiff[q2 * K + q] = g_new - g_old;
      }
      // (A3) Y = V B0 (register mode: from the tiles, with the window columns' magnitudes)
      if constexpr (RT > 0) {
        regb_window<RT>(breg, vcur, ldv, ywin, nP, Kw, nt, lane, wave);
        regb_magnitudes<RT>(breg, vcur, ldv, rmag, k0, Kw, n, nt, lane, wave);
      } else {
        gemm_window<T, MF>(vwin, Bm, ldb, ywin, Kw, n, nP, tid);
      }
      __syncthreads();
      if (sizeof(T) == 4) {
        // mixed: |v_q^T B0|^2 partials (row q of Y), for the inverse-error part of the guard band
        const int q = tid / tpq, s = tid - q * tpq;
        double t2 = 0.0;
        if (q < Kw)
          for (int c = s; c < n; c += tpq) {
            const double y = (double)ywin[(size_t)q * nP + c];
            t2 += y * y;
          }
        tnp[tid] = t2;
        __syncthreads();
      }

      // (B) the moves of the window, in order, by one wave.  Lane q keeps move q's Jastrow
      // change (partners at their positions before the window, in-window partners too) and
      // row q of the window block yk = Y[:, k0 .. k0 + Kw).  An accepted move q eliminates
      // its column from the later rows (the Sherman-Morrison update restricted to the
      // window's own columns), so each ratio is read, not recomputed: R_q = yk[q][q].
      if (wave == seq_wave) {
        if (lane == 0) sm_stop = -1;
        double Fq = 0.0, Sq = 0.0, Eq = 0.0, Tq = 0.0;
        if (lane < Kw) {
          for (int s = 0; s < tpq; ++s) Fq += red[lane * tpq + s];
          if (sizeof(T) == 4) {
            if (RT > 0) Sq = rmag[lane];
            else
              for (int s = 0; s < tpq; ++s) Sq += rmag[lane * tpq + s];
            for (int s = 0; s < tpq; ++s) Tq += tnp[lane * tpq + s];
            Tq = sqrt(Tq);
          }
          for (int j = 0; j < Kw; ++j) {
            const double gj = gold[j * K + lane];
            Fq += j != lane ? gj : 0.0;
          }
        }
        wave_sync_lds();   // gold is consumed: its storage takes yk
        if (lane < Kw)
          for (int j = 0; j < Kw; ++j) yk[lane * ldy + j] = (double)ywin[(size_t)lane * nP + k0 + j];
        // mixed precision: an FP32 exponential is well inside the guard band
        auto jexp = [](double x) { return sizeof(T) == 4 ? (double)__expf((float)x) : exp(x); };
        // lane q: its move's acceptance uniform and the exponential of its current Jastrow
        // change (kept current as earlier moves are accepted)
        const double uq = lane < Kw ? sprop[4 * (k0 + lane) + 3] : 0.0;
        double exq = lane < Kw ? jexp(2.0 * Fq) : 0.0;
        double racc = 1.0;      // lane q: R of move q once accepted
        uint64_t amask = 0;     // accepted moves of the window
        uint64_t dmask = 0;     // decided moves of the window (accepted or rejected)
        // guard band terms that do not change over the window (mixed precision)
        const double uf = 5.9604644775390625e-08;   // 2^-24
        const double band0 = sizeof(T) == 4 ? P.tie_guard + 4.0 * uf : P.tie_guard;
        const double nuf2 = 2.0 * (n + 1) * uf;
        wave_sync_lds();
        int m = 0;
        for (int q = 0; q < Kw; ++q) {
          const double R = yk[q * ldy + q];
          // one reciprocal serves the guard band and the elimination below; it is formed
          // while the lane reads complete
          const double invR = 1.0 / R;
          const double u = readlane_d(uq, q);
          const double ex = readlane_d(exq, q);
          // later lanes: their exponential should move q be accepted, formed ahead of the
          // decision
          const bool later = lane > q && lane < Kw;
          const double gq = later ? gdiff[q * K + lane] : 0.0;
          const double ex_acc = later ? jexp(2.0 * (Fq + gq)) : 0.0;
          const double p32 = R * R * ex;
          // guard band: the relative tie guard, widened by a bound on the FP32 rounding of R:
          // n + 1 unit roundoffs (the length-n product and the cast of B0) of the magnitude of
          // the terms that formed R, sum_l |v_l B0[l][k]| plus the eliminated window terms --
          // ratios that cancel heavily are re-decided in FP64
          double band = band0;
          if (sizeof(T) == 4)
            band += (nuf2 * (readlane_d(Sq, q) + readlane_d(Eq, q)) + readlane_d(ecq, q) * readlane_d(Tq, q)) *
                    fabs(invR);
          if (sizeof(T) == 4 && fabs(u - p32) <= band * p32) {
            // near tie in FP32: end the window here; the move is re-decided in FP64 below
            const double dJ = readlane_d(Fq, q);
            if (lane == 0) { sm_stop = q; sm_dj = dJ; }
            break;
          }
          if (u < p32) {
            const double Tacc = sizeof(T) == 4 ? readlane_d(Tq, q) : 0.0;
            if (lane > q && lane < Kw) {
              double* ykl = yk + lane_now() * ldy;   // this lane's row
              const double f = ykl[q] * invR;
              if (sizeof(T) == 4) {
                Eq += fabs(f * yk[q * ldy + lane_now()]);
                Tq += fabs(f) * Tacc;   // row q's new v^T B is its old one minus f times move q's
              }
              // eight columns at a time: all loads before the stores, so they overlap.  The
              // loads are unconditional (a guarded load becomes a branch of its own): columns
              // past Kw read at most 7 entries beyond the row, inside the LDS block that
              // follows yk, and are never stored.
              for (int j0 = q + 1; j0 < Kw; j0 += 8) {
                double pv[8], rv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                  pv[e] = yk[q * ldy + j0 + e];
                  rv[e] = ykl[j0 + e];
                }
#pragma unroll
                for (int e = 0; e < 8; ++e)
                  if (j0 + e < Kw) ykl[j0 + e] = rv[e] - f * pv[e];
              }
              Fq += gq;
              exq = ex_acc;
            }
            ++m;
            ++nacc;
            racc = lane == q ? R : racc;
            amask |= 1ull << q;
            if (R < 0.0) sgn = -sgn;
          }
          dmask |= 1ull << q;
          wave_sync_lds();
        }
        if ((dmask >> lane) & 1ull) {
          // the decided moves' bookkeeping, lane q for move q, once the window's decisions are
          // made: accepted moves take their place in the flush lists (in move order) and the
          // electron its new position
          const int kq = k0 + lane, iq = off + kq;
          if ((amask >> lane) & 1ull) {
            const int slot = __popcll(amask & ((1ull << lane) - 1ull));
            plist[slot] = kq;
            qlist[slot] = lane;
            spos[3 * iq] = sprop[4 * kq];
            spos[3 * iq + 1] = sprop[4 * kq + 1];
            spos[3 * iq + 2] = sprop[4 * kq + 2];
            scur[kq] = (uint8_t)(1 - scur[kq]);
            sacc[kq] = 1;
          } else {
            sacc[kq] = 0;
          }
        }
        {
          // log|R| of the accepted moves: all lanes at once, added in move order
          const double lg = log(fabs(racc));
          for (int q = 0; q < Kw; ++q)
            if ((amask >> q) & 1ull) logd += readlane_d(lg, q);
        }
        if (lane == 0) sm_m = m;
      } else if (RT > 0 && k0 + Kw < n) {
        // register mode: meanwhile the other waves fetch the next window's rows (for the window
        // that follows when no near tie cuts this one short; the moves only change this window's
        // buffer flags)
        const int nk0 = k0 + Kw, nkw = (n - nk0) < K ? (n - nk0) : K;
        const int pw = wave < seq_wave ? wave : wave - 1;
        load_rows(vpre, item0, nk0, nkw, nt, n, scur, pw * 64 + lane, (kWaves - 1) * 64);
      }
      pre_k0 = (RT > 0 && k0 + Kw < n) ? k0 + Kw : -1;
      __syncthreads();

      // (C) flush: B = B0 - B0[:, P] C^-1 (Y[Q, :] - E_P^T), C = Y[Q, P].  C^-1 by
      // Gauss-Jordan elimination without pivoting over the whole workgroup (its pivots are
      // the accepted ratios, all nonzero), each step from one buffer into the other; the
      // storage of gold and gdiff is free after (B).
      const int m = sm_m;
      if (m > 0) {
        const int mP = (m + 3) & ~3;
        double* ga = reinterpret_cast<double*>(smem + lay.gold);
        double* gb = reinterpret_cast<double*>(smem + lay.gdiff);
        for (int idx = tid; idx < m * m; idx += kBlock) {
          const int a = idx / m, b = idx - a * m;
          ga[a * K + b] = (double)ywin[(size_t)qlist[a] * nP + plist[b]];
        }
        __syncthreads();
        // the elimination in one wave: its steps are ordered by wave-level LDS syncs, with no
        // workgroup barrier per pivot (the other waves wait once, below)
        if (wave == 0) {
          // lane (j0, i0) = (lane % 16, lane / 16) takes the entries (i0 + 4 a, j0 + 16 b)
          double* a0 = ga;
          double* b1 = gb;
          for (int pv = 0; pv < m; ++pv) {
            const double inv = 1.0 / a0[pv * K + pv];
            for (int j = lane & 15; j < m; j += 16) {
              const double apj = a0[pv * K + j];
              for (int i = lane >> 4; i < m; i += 4) {
                const double aip = a0[i * K + pv];
                b1[i * K + j] = i == pv ? (j == pv ? inv : apj * inv)
                                        : (j == pv ? -aip * inv : a0[i * K + j] - aip * apj * inv);
              }
            }
            wave_sync_lds();
            double* t = a0; a0 = b1; b1 = t;
          }
        }
        __syncthreads();
        const double* cinv = (m & 1) ? gb : ga;   // after m steps, from one buffer into the other
        // register mode: Z is read up to the tiles' 16 nt columns, zero past n
        const int nz = RT > 0 ? 16 * nt : n;
        if constexpr (MF) {
          capacitance_z<T>(cinv, K, ywin, nP, qlist, plist, m, mP, n, nz, zwin, lane, wave);
        } else {
          for (int idx = tid; idx < mP * nz; idx += kBlock) {
            const int r = idx / nz, c = idx - r * nz;
            double acc = 0.0;
            if (r < m && c < n)
              for (int l = 0; l < m; ++l)
                acc += cinv[r * K + l] * ((double)ywin[(size_t)qlist[l] * nP + c] - (c == plist[l] ? 1.0 : 0.0));
            zwin[(size_t)r * nP + c] = (T)acc;
          }
        }
        __syncthreads();   // Y is dead from here: U takes its storage
        if constexpr (RT > 0) {
          regb_columns<RT>(breg, ubuf, nP + 1, plist, m, mP, nt, lane, wave, tid);
          __syncthreads();
          regb_flush<RT>(breg, ubuf, nP + 1, zwin, nP, mP, nt, lane, wave);
          __syncthreads();   // U and Z are read before the next window writes their storage
        } else {
          for (int idx = tid; idx < n * mP; idx += kBlock) {
            const int l = idx / mP, r = idx - l * mP;
            ubuf[(size_t)l * K + r] = (r < m) ? Bm[(size_t)l * ldb + plist[r]] : T(0);
          }
          __syncthreads();
          constexpr int kVec = 16 / sizeof(T);
          if (!BLDS && (n & 3) == 0 && (n % kVec) == 0 && (ldb % kVec) == 0 &&
              (reinterpret_cast<uintptr_t>(Bm) & 15) == 0)
            flush_global<T>(Bm, ldb, ubuf, K, zwin, nP, n, mP, tid);
          else
            gemm_flush<T, MF>(Bm, ldb, ubuf, K, zwin, nP, n, mP, tid);
          __syncthreads();
        }
      }
      // (D) a move stopped at a near tie (mixed precision): FP64 decision against the
      // now current inverse, Sherman-Morrison update if accepted
      const int stop = sm_stop;
      if (stop >= 0) {
        const int kq = k0 + stop, iq = off + kq;
        const size_t it = item0 + kq;
        const T* vg = Wk.vgl + ((size_t)(1 - scur[kq]) * P.W * N + it) * Wk.vstride;
        const double* v64 = Wk.val64 + ((size_t)(1 - scur[kq]) * P.W * N + it) * P.S;
        double R64;
        if constexpr (RT > 0) {
          // register mode: the row vector t = v^T A^-1 refined in FP64 against the FP64 Slater
          // matrix A, t <- t + (v - t^T A) B from t = v^T B (each step multiplies the error by
          // I - A B); R = t[k].  tf keeps the FP32 v^T B of the update.
          float* tf = reinterpret_cast<float*>(ywin);   // free after the flush
          for (int l = tid; l < 16 * nt; l += kBlock) sgrow[l] = l < n ? vg[l] : T(0);
          __syncthreads();
          regb_rowvec<RT>(breg, sgrow, sgx, false, n, nt, lane, wave);
          __syncthreads();
          for (int c = tid; c < n; c += kBlock) tf[c] = (float)sgx[c];
          for (int step = 0; step < 3; ++step) {
            for (int l = tid; l < 16 * nt; l += kBlock) {
              double a = 0.0;
              if (l < n) {
                a = v64[l];
#pragma unroll 8
                for (int j = 0; j < n; ++j)
                  a -= sgx[j] * Wk.val64[((size_t)scur[j] * P.W * N + item0 + j) * P.S + l];
              }
              sgr[l] = a;
            }
            __syncthreads();
            regb_rowvec<RT>(breg, sgr, sgx, true, n, nt, lane, wave);
            __syncthreads();
          }
          R64 = sgx[kq];
        } else {
          for (int l = tid; l < n; l += kBlock) sgrow[l] = vg[l];
          R64 = refined_ratio<T>(P, Wk, Bm, ldb, n, item0, scur, v64, kq, sgx, sgr, red, tid);
        }
        const double dJ = sm_dj;
        const double u = sprop[4 * kq + 3];
        ++nguard;
        if (u < R64 * R64 * exp(2.0 * dJ)) {
          if constexpr (RT > 0) {
            float* tf = reinterpret_cast<float*>(ywin);
            float* col = reinterpret_cast<float*>(zwin);
            regb_column<RT>(breg, col, kq, nt, lane, wave);
            __syncthreads();
            regb_rank1<RT>(breg, col, tf, 1.0f / tf[kq], kq, n, nt, lane, wave);
          } else {
            // t = v^T B (FP32), column kq saved, then B -= B[:, kq] (t - e_kq) / t_kq
            T* st = ywin;              // free after the flush
            T* scol = zwin;
            for (int m = tid; m < n; m += kBlock) {
              T acc = T(0);
              for (int l = 0; l < n; ++l) acc += sgrow[l] * Bm[(size_t)l * ldb + m];
              st[m] = acc;
              scol[m] = Bm[(size_t)m * ldb + kq];
            }
            __syncthreads();
            const T invR = T(1) / st[kq];
            __syncthreads();
            for (int idx = tid; idx < n * n; idx += kBlock) {
              const int l = idx / n, m = idx - l * n;
              Bm[(size_t)l * ldb + m] -= scol[l] * invR * (st[m] - (m == kq ? T(1) : T(0)));
            }
          }
          if (tid == 0) {
            spos[3 * iq] = sprop[4 * kq];
            spos[3 * iq + 1] = sprop[4 * kq + 1];
            spos[3 * iq + 2] = sprop[4 * kq + 2];
            scur[kq] = (uint8_t)(1 - scur[kq]);
            sacc[kq] = 1;
          }
          ++nacc;
          logd += log(fabs(R64));
          if (R64 < 0.0) sgn = -sgn;
        } else if (tid == 0) {
          sacc[kq] = 0;
        }
        __syncthreads();
        k0 = kq + 1;
      } else {
        k0 += Kw;
      }
    }
    if constexpr (RT > 0) regb_store<RT>(breg, Bg, reinterpret_cast<float*>(ywin), n, nt, lane, wave, tid);
    __syncthreads();
    for (int q = tid; q < n; q += kBlock) {
      Wk.cur[item0 + q] = scur[q];
      Wk.acc[item0 + q] = sacc[q];
    }
    if (tid == seq_tid) {   // the sequential wave holds the complete log|D|, sign and counts
      Wk.logdet[2 * w + sp] = logd;
      Wk.sign[2 * w + sp] = sgn;
    }
    if (BLDS) {
      for (int q = tid; q < n * n; q += kBlock) {
        const int l = q / n;
        Bg[q] = sB[l * ldl + (q - l * n)];
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < 3 * N; j += kBlock) Wk.pos[(size_t)w * 3 * N + j] = spos[j];
  if (tid == seq_tid) {
    Wk.nacc[w] = nacc;
    Wk.nguard[w] += nguard;
    if (Wk.eta_age) Wk.eta_age[w] += 1u;
    if (Wk.fb && Wk.fb_sel == 1) Wk.pstat[2 * w + 1] += 1u;
    if (w == 0) *Wk.sweep_ctr += 1u;   // read by the next sweep's gather
  }
}

template <typename T, bool BLDS, bool MF>
__global__ __launch_bounds__(kBlock, 2) void k_chain_delayed(SysParams P, Walkers<T> Wk, int K, int ldl) {
  chain_delayed_walker<T, BLDS, MF, 0>(P, Wk, blockIdx.x, K, ldl);
}

// The inverse in registers (FP32, spin blocks up to 16 kRegTiles), two workgroups per compute
// unit: the compiler then keeps the kernel within 256 registers per lane and moves a few values
// to scratch, which costs less than one walker per compute unit with no latency hidden.
constexpr int kRegTiles = 12;
__global__ __launch_bounds__(kBlock, 2) void k_chain_delayed_reg(SysParams P, Walkers<float> Wk, int K, int ldl) {
  chain_delayed_walker<float, false, true, kRegTiles>(P, Wk, blockIdx.x, K, ldl);
}

// Several systems in one launch: block b is walker bmap[b].y of system bmap[b].x.
template <typename T, bool BLDS, bool MF>
__global__ __launch_bounds__(kBlock, 2) void k_chain_delayed_batched(const SysDev<T>* __restrict__ sd,
                                                                  const int2* __restrict__ bmap) {
  __shared__ SysDev<T> s;
  const int2 m = bmap[blockIdx.x];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(sd + m.x);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&s);
    for (int q = threadIdx.x; q < (int)(sizeof(SysDev<T>) / 4); q += kBlock) dst[q] = src[q];
  }
  __syncthreads();
  chain_delayed_walker<T, BLDS, MF, 0>(s.P, s.W, m.y, s.K, s.ldl);
}

static int lds_budget_d() {
  static int budget = -1;
  if (budget < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      budget = v;
    else
      budget = 163840;   // gfx950: 160 KiB of LDS per workgroup
  }
  return budget;
}

template <typename T, bool BLDS, bool MF>
static hipError_t launch_delayed_variant(const SysParams& P, const Walkers<T>& Wk, int K, hipStream_t st,
                                         size_t bytes, int ldl) {
  if (bytes > 65536) {
    const hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_chain_delayed<T, BLDS, MF>));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_chain_delayed<T, BLDS, MF>), dim3(P.W), dim3(kBlock), bytes, st, P, Wk, K, ldl);
  return hipGetLastError();
}

bool delayed_feasible(const SysParams& P, size_t tsize, int K) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  return dlayout(P.N, nmax, P.n_ions, nmax | 1, tsize, false, K).total + sizeof(Jastrow) +
             sizeof(SysDev<double>) <= (size_t)lds_budget_d();
}

size_t delayed_lds_bytes(const SysParams& P, size_t tsize, bool b_in_lds, int K) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  return dlayout(P.N, nmax, P.n_ions, nmax | 1, tsize, b_in_lds, K).total;
}

// Whether the register-resident variant takes a chain: FP32, matrix cores, spin blocks up to
// 16 kRegTiles and windows up to 32.  It runs where the inverse does not fit the LDS, or
// everywhere it can with QMC_CHAIN_REGISTER_INVERSE=1 (lets the tests cover it on small systems);
// QMC_CHAIN_REGISTER_INVERSE=0 switches it off.
static bool use_register_chain(const SysParams& P, size_t tsize, int K, int use_mfma, bool lds_fits) {
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  // (K >= 8: the window's Y and Z storage holds the 16-row staging slab)
  if (tsize != sizeof(float) || !use_mfma || nmax > 16 * kRegTiles || K > 32 || K < 8) return false;
  const char* e = getenv("QMC_CHAIN_REGISTER_INVERSE");
  if (e && e[0] == '0') return false;
  if (e && e[0] == '1') return true;
  return !lds_fits;
}

template <typename T>
hipError_t launch_chain_delayed(const SysParams& P, const Walkers<T>& Wk, int K, int use_mfma, hipStream_t st) {
  // K >= 4 keeps the flush's padded rank (a multiple of 4) within the K-wide buffers
  if (K < 4 || K > kMaxWindow || (K & (K - 1))) return hipErrorInvalidValue;
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  const int ldl = nmax | 1;
  const size_t with_b = dlayout(P.N, nmax, P.n_ions, ldl, sizeof(T), true, K).total + sizeof(Jastrow);
  const size_t without_b = dlayout(P.N, nmax, P.n_ions, ldl, sizeof(T), false, K).total + sizeof(Jastrow);
  const char* fg = getenv("QMC_CHAIN_GLOBAL_INVERSE");
  const bool force_global = fg && fg[0] == '1';
  const size_t budget = (size_t)lds_budget_d();
  const size_t with_pre = dlayout(P.N, nmax, P.n_ions, ldl, sizeof(T), false, K, true).total + sizeof(Jastrow);
  if (sizeof(T) == sizeof(float) && !force_global && with_pre <= budget &&
      use_register_chain(P, sizeof(T), K, use_mfma, with_b <= budget)) {
    const size_t bytes = with_pre - sizeof(Jastrow);
    if (bytes > 65536) {
      const hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_chain_delayed_reg));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_chain_delayed_reg, dim3(P.W), dim3(kBlock), bytes, st, P,
                       *reinterpret_cast<const Walkers<float>*>(&Wk), K, ldl);
    return hipGetLastError();
  }
  if (!force_global && with_b <= budget) {
    const size_t bytes = with_b - sizeof(Jastrow);
    return use_mfma ? launch_delayed_variant<T, true, true>(P, Wk, K, st, bytes, ldl)
                    : launch_delayed_variant<T, true, false>(P, Wk, K, st, bytes, ldl);
  }
  if (without_b > budget) return hipErrorInvalidValue;
  const size_t bytes = without_b - sizeof(Jastrow);
  return use_mfma ? launch_delayed_variant<T, false, true>(P, Wk, K, st, bytes, ldl)
                  : launch_delayed_variant<T, false, false>(P, Wk, K, st, bytes, ldl);
}

template <typename T, bool BLDS, bool MF>
static hipError_t launch_delayed_batched_variant(const SysDev<T>* sd, const int2* bmap, int n_blocks, size_t lds,
                                                 hipStream_t st) {
  if (lds > 65536) {
    const hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_chain_delayed_batched<T, BLDS, MF>));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_chain_delayed_batched<T, BLDS, MF>), dim3(n_blocks), dim3(kBlock), lds, st, sd, bmap);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_chain_delayed_batched(const SysDev<T>* sd, const int2* bmap, int n_blocks, bool b_in_lds,
                                        int use_mfma, size_t lds, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (lds + sizeof(Jastrow) + sizeof(SysDev<T>) > (size_t)lds_budget_d()) return hipErrorInvalidValue;
  if (b_in_lds)
    return use_mfma ? launch_delayed_batched_variant<T, true, true>(sd, bmap, n_blocks, lds, st)
                    : launch_delayed_batched_variant<T, true, false>(sd, bmap, n_blocks, lds, st);
  return use_mfma ? launch_delayed_batched_variant<T, false, true>(sd, bmap, n_blocks, lds, st)
                  : launch_delayed_batched_variant<T, false, false>(sd, bmap, n_blocks, lds, st);
}

template hipError_t launch_chain_delayed<double>(const SysParams&, const Walkers<double>&, int, int, hipStream_t);
template hipError_t launch_chain_delayed<float>(const SysParams&, const Walkers<float>&, int, int, hipStream_t);
template hipError_t launch_chain_delayed_batched<double>(const SysDev<double>*, const int2*, int, bool, int, size_t,
                                                         hipStream_t);
template hipError_t launch_chain_delayed_batched<float>(const SysDev<float>*, const int2*, int, bool, int, size_t,
                                                        hipStream_t);

template <typename T>
static hipError_t delayed_lds_limits_t() {
  const void* ks[] = {reinterpret_cast<const void*>(&k_chain_delayed_reg),
                      reinterpret_cast<const void*>(&k_chain_delayed<T, true, true>),
                      reinterpret_cast<const void*>(&k_chain_delayed<T, true, false>),
                      reinterpret_cast<const void*>(&k_chain_delayed<T, false, true>),
                      reinterpret_cast<const void*>(&k_chain_delayed<T, false, false>),
                      reinterpret_cast<const void*>(&k_chain_delayed_batched<T, true, true>),
                      reinterpret_cast<const void*>(&k_chain_delayed_batched<T, true, false>),
                      reinterpret_cast<const void*>(&k_chain_delayed_batched<T, false, true>),
                      reinterpret_cast<const void*>(&k_chain_delayed_batched<T, false, false>)};
  for (const void* k : ks) {
    const hipError_t e = allow_dynamic_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t delayed_lds_limits() {
  const hipError_t e = delayed_lds_limits_t<double>();
  return e != hipSuccess ? e : delayed_lds_limits_t<float>();
}

}  // namespace qmc
