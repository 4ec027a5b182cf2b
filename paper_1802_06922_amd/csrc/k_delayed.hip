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
  size_t pos, prop, ions, red, rmag, tn, gold, gdiff, cur, acc, plist, qlist, vwin, ywin, zwin, gx, gr, grow, b,
      total;
};

__host__ __device__ inline int round16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline DLayout dlayout(int N, int nmax, int n_ions, int ldl, size_t ts, bool b_in_lds,
                                           int K) {
  DLayout L;
  const int nP = round16(nmax);
  size_t o = 0;
  auto al = [&](size_t a) { o = (o + a - 1) & ~(a - 1); };
  L.pos = o; o += sizeof(double) * 3 * N;
  L.prop = o; o += sizeof(double) * 4 * nmax;
  L.ions = o; o += (n_ions <= kLdsIonsD) ? sizeof(double) * 4 * n_ions : 0;
  L.red = o; o += sizeof(double) * kBlock;
  L.rmag = o; o += (ts == 4) ? sizeof(double) * kBlock : 0;   // mixed: |v| . |B0[:, k]| partials
  L.tn = o; o += (ts == 4) ? sizeof(double) * kBlock : 0;     // mixed: |v^T B0|^2 partials
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
  L.ywin = o; o += ts * (size_t)K * nP;
  al(16);
  L.zwin = o; o += ts * (size_t)K * nP;
  L.vwin = L.zwin;
  al(16);
  L.gx = o; o += (ts == 4) ? sizeof(double) * nmax : 0;   // FP64 re-decision scratch (mixed)
  L.gr = o; o += (ts == 4) ? sizeof(double) * nmax : 0;
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

// Orders this wave's LDS writes before its later LDS reads (lanes read what
// other lanes of the same wave wrote).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
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
    const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
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

// B[l][c] -= sum_r U[l][r] Z[r][c] for l, c < n, r < mP (U, Z zero-padded to mP).
template <typename T, bool MF>
__device__ __forceinline__ void gemm_flush(T* B, int ldb, const T* U, int ldu, const T* Z, int nP, int n,
                                           int mP, int tid) {
  if (MF) {
    typedef Mfma<T> M;
    constexpr int kGroup = Group<T>::n;
    const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
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

template <typename T, bool BLDS, bool MF>
__device__ __forceinline__ void chain_delayed_walker(const SysParams& P, const Walkers<T>& Wk, int w, int K,
                                                     int ldl) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Jastrow sj;
  __shared__ int sm_m, sm_stop;
  __shared__ double sm_dj;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (chain_skips(Wk, w)) return;
  const int N = P.N, nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn, nP = round16(nmax);
  const DLayout lay = dlayout(N, nmax, P.n_ions, ldl, sizeof(T), BLDS, K);
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
  const int ldy = K + 1;        // row stride of yk: the lanes' rows start in different banks
  // the wave that runs the moves in sequence rotates with the workgroup index, so that the
  // sequential phases of workgroups sharing a compute unit fall on different SIMDs
  const int seq_wave = (int)(blockIdx.x & (kWaves - 1)), seq_tid = seq_wave * 64;

  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.jas);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&sj);
    for (int q = tid; q < (int)(sizeof(Jastrow) / 4); q += kBlock) dst[q] = src[q];
  }
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
    __syncthreads();   // the block's proposals, buffer flags and inverse are staged before any use

    for (int k0 = 0; k0 < n;) {
      const int Kw = (n - k0) < K ? (n - k0) : K;
      // (A1) the window's proposal rows
      for (int idx = tid; idx < Kw * n; idx += kBlock) {
        const int q = idx / n, l = idx - q * n;
        const size_t it = item0 + k0 + q;
        vwin[(size_t)q * nP + l] = Wk.vgl[((size_t)(1 - scur[k0 + q]) * P.W * N + it) * Wk.vstride + l];
      }
      __syncthreads();
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
          auto range = [&](const Radial& R, int lo, int hi, const double* c, int stride) {
            for (int j = lo + s; j < hi; j += tpq) {
              const double* cj = c + (size_t)stride * j;
              part += radial_value(R, dist(px, py, pz, cj[0], cj[1], cj[2], L, invL)) -
                      radial_value(R, dist(ox, oy, oz, cj[0], cj[1], cj[2], L, invL));
            }
          };
          const int ooff = up_block ? P.n_up : 0, no = up_block ? P.n_dn : P.n_up;
          range(sj.same, off, off + k0, spos, 3);
          range(sj.same, off + k0 + Kw, off + n, spos, 3);
          range(sj.opp, ooff, ooff + no, spos, 3);
          range(sj.ei, 0, P.n_ions, ions, 4);
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
        if (sizeof(T) == 4) {
          // magnitude of the ratio's terms, sum_l |v_l| |B0[l][k]|, which bounds the FP32
          // rounding of the ratio (mixed precision guard band)
          double mag = 0.0;
          if (q < Kw)
            for (int l = s; l < n; l += tpq)
              mag += fabs((double)vwin[(size_t)q * nP + l]) * fabs((double)Bm[(size_t)l * ldb + k0 + q]);
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
      // (A3) Y = V B0
      gemm_window<T, MF>(vwin, Bm, ldb, ywin, Kw, n, nP, tid);
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
        wave_sync_lds();
        int m = 0;
        for (int q = 0; q < Kw; ++q) {
          const int kq = k0 + q, iq = off + kq;
          const double R = yk[q * ldy + q];
          const double dJ = readlane_d(Fq, q);
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
          double band = P.tie_guard;
          if (sizeof(T) == 4) {
            const double uf = 5.9604644775390625e-08;   // 2^-24
            const double err = (n + 1) * uf * (readlane_d(Sq, q) + readlane_d(Eq, q));
            band += 2.0 * err / fabs(R) + 4.0 * uf + inverse_error_term(Wk, w, sp, n, readlane_d(Tq, q), R);
          }
          if (sizeof(T) == 4 && fabs(u - p32) <= band * p32) {
            // near tie in FP32: end the window here; the move is re-decided in FP64 below
            if (lane == 0) { sm_stop = q; sm_dj = dJ; }
            break;
          }
          if (u < p32) {
            const double Tacc = sizeof(T) == 4 ? readlane_d(Tq, q) : 0.0;
            if (lane > q && lane < Kw) {
              const double f = yk[lane * ldy + q] / R;
              if (sizeof(T) == 4) {
                Eq += fabs(f * yk[q * ldy + lane]);
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
                  rv[e] = yk[lane * ldy + j0 + e];
                }
#pragma unroll
                for (int e = 0; e < 8; ++e)
                  if (j0 + e < Kw) yk[lane * ldy + j0 + e] = rv[e] - f * pv[e];
              }
              Fq += gq;
              exq = ex_acc;
            }
            if (lane == 0) {
              plist[m] = kq;
              qlist[m] = q;
              spos[3 * iq] = sprop[4 * kq];
              spos[3 * iq + 1] = sprop[4 * kq + 1];
              spos[3 * iq + 2] = sprop[4 * kq + 2];
              scur[kq] = (uint8_t)(1 - scur[kq]);
              sacc[kq] = 1;
            }
            ++m;
            ++nacc;
            racc = lane == q ? R : racc;
            amask |= 1ull << q;
            if (R < 0.0) sgn = -sgn;
          } else if (lane == 0) {
            sacc[kq] = 0;
          }
          wave_sync_lds();
        }
        {
          // log|R| of the accepted moves: all lanes at once, added in move order
          const double lg = log(fabs(racc));
          for (int q = 0; q < Kw; ++q)
            if ((amask >> q) & 1ull) logd += readlane_d(lg, q);
        }
        if (lane == 0) sm_m = m;
      }
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
        for (int pv = 0; pv < m; ++pv) {
          const double inv = 1.0 / ga[pv * K + pv];
          for (int idx = tid; idx < m * m; idx += kBlock) {
            const int i = idx / m, j = idx - i * m;
            const double aip = ga[i * K + pv], apj = ga[pv * K + j];
            gb[i * K + j] = i == pv ? (j == pv ? inv : apj * inv)
                                    : (j == pv ? -aip * inv : ga[i * K + j] - aip * apj * inv);
          }
          __syncthreads();
          double* t = ga; ga = gb; gb = t;
        }
        const double* cinv = ga;
        for (int idx = tid; idx < mP * n; idx += kBlock) {
          const int r = idx / n, c = idx - r * n;
          double acc = 0.0;
          if (r < m)
            for (int l = 0; l < m; ++l)
              acc += cinv[r * K + l] * ((double)ywin[(size_t)qlist[l] * nP + c] - (c == plist[l] ? 1.0 : 0.0));
          zwin[(size_t)r * nP + c] = (T)acc;
        }
        __syncthreads();   // Y is dead from here: U takes its storage
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
      // (D) a move stopped at a near tie (mixed precision): FP64 decision against the
      // now current inverse, Sherman-Morrison update if accepted
      const int stop = sm_stop;
      if (stop >= 0) {
        const int kq = k0 + stop, iq = off + kq;
        const size_t it = item0 + kq;
        const T* vg = Wk.vgl + ((size_t)(1 - scur[kq]) * P.W * N + it) * Wk.vstride;
        for (int l = tid; l < n; l += kBlock) sgrow[l] = vg[l];
        const double* v64 = Wk.val64 + ((size_t)(1 - scur[kq]) * P.W * N + it) * P.S;
        const double R64 = refined_ratio<T>(P, Wk, Bm, ldb, n, item0, scur, v64, kq, sgx, sgr, red, tid);
        const double dJ = sm_dj;
        const double u = sprop[4 * kq + 3];
        ++nguard;
        if (u < R64 * R64 * exp(2.0 * dJ)) {
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
  chain_delayed_walker<T, BLDS, MF>(P, Wk, blockIdx.x, K, ldl);
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
  chain_delayed_walker<T, BLDS, MF>(s.P, s.W, m.y, s.K, s.ldl);
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
  const void* ks[] = {reinterpret_cast<const void*>(&k_chain_delayed<T, true, true>),
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
