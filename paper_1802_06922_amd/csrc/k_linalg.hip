// k_linalg.hip -- full FP64 rebuild of every Slater-matrix inverse.
//
// A[k][l] = phi_l(r_k) is assembled from the current value rows, inverted in
// place by Gauss-Jordan elimination with partial (row) pivoting in FP64, and
// the result B = A^-1 (B[l][k], row = orbital) is stored in the handle's
// precision together with log|det A| and its sign.  This is the full
// recompute that bounds the drift of the rank-one (or delayed) updates; the
// paper keeps such high-precision steps in double even in its mixed-precision
// builds (section "Code structure": precision is a build parameter).
//
// One workgroup per (walker, spin).  The matrix lives in an FP64 scratch
// buffer; the pivot column is staged in LDS.
#include "qmc_kernels.hpp"

namespace qmc {

constexpr int kMaxSpin = 1024;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rebuild(SysParams P, Walkers<T> Wk, double* scratch,
                                                    double* drift, const uint32_t* sel, uint32_t sel_value) {
  __shared__ double scol[kMaxSpin];
  __shared__ int perm[kMaxSpin];
  __shared__ double rv[kWaves];
  __shared__ int ri[kWaves];
  const int w = blockIdx.x >> 1, sp = blockIdx.x & 1, tid = threadIdx.x;
  const int lane = tid & 63, wave = wave_of(tid);
  const int n = sp ? P.n_dn : P.n_up, off = sp ? P.n_up : 0;
  const int N = P.N;
  if (sel && sel[w] != sel_value) return;
  if (n == 0) {
    if (tid == 0) {
      if (drift) drift[2 * w + sp] = Wk.logdet[2 * w + sp];
      Wk.logdet[2 * w + sp] = 0.0;
      Wk.sign[2 * w + sp] = 1;
    }
    return;
  }
  const size_t boff = (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
  double* a = scratch + boff;
  double amax = 0.0;
  for (int q = tid; q < n * n; q += kBlock) {
    const int k = q / n, l = q - k * n;
    const size_t item = (size_t)w * N + off + k;
    const int cb = Wk.cur[item] ^ Wk.row_flip;
    a[q] = Wk.val64 ? Wk.val64[((size_t)cb * P.W * N + item) * P.S + l]
                    : (double)Wk.vgl[((size_t)cb * P.W * N + item) * kComp * P.S + l];
    amax = fmax(amax, fabs(a[q]));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
  if (lane == 0) rv[wave] = amax;
  __syncthreads();
  amax = fmax(fmax(rv[0], rv[1]), fmax(rv[2], rv[3]));
  // a pivot this small relative to the largest entry means a numerically singular matrix
  const double tiny = 1e-14 * amax;
  __syncthreads();
  double logabs = 0.0;
  int sgn = 1;
  bool singular = false;
  for (int k = 0; k < n; ++k) {
    // pivot: largest |a[i][k]|, i >= k (smallest index on ties)
    double best = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += kBlock) {
      const double v = fabs(a[(size_t)i * n + k]);
      if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { rv[wave] = best; ri[wave] = bi; }
    __syncthreads();
    best = rv[0];
    bi = ri[0];
    for (int q = 1; q < kWaves; ++q)
      if (rv[q] > best || (rv[q] == best && ri[q] < bi)) { best = rv[q]; bi = ri[q]; }
    if (!(best > tiny) || !isfinite(best)) { singular = true; break; }
    if (bi != k) {
      for (int j = tid; j < n; j += kBlock) {
        const double x = a[(size_t)k * n + j];
        a[(size_t)k * n + j] = a[(size_t)bi * n + j];
        a[(size_t)bi * n + j] = x;
      }
      sgn = -sgn;
    }
    if (tid == 0) perm[k] = bi;
    __syncthreads();
    for (int i = tid; i < n; i += kBlock) scol[i] = a[(size_t)i * n + k];
    __syncthreads();
    const double piv = scol[k];
    const double pinv = 1.0 / piv;
    logabs += log(fabs(piv));
    if (piv < 0.0) sgn = -sgn;
    for (int j = tid; j < n; j += kBlock) a[(size_t)k * n + j] = (j == k) ? pinv : a[(size_t)k * n + j] * pinv;
    __syncthreads();
    for (int i = wave; i < n; i += kWaves) {
      if (i == k) continue;
      const double f = scol[i];
      double* ai = a + (size_t)i * n;
      const double* ak = a + (size_t)k * n;
      for (int j = lane; j < n; j += 64) ai[j] = ((j == k) ? 0.0 : ai[j]) - f * ak[j];
    }
    __syncthreads();
  }
  if (!singular) {
    for (int k = n - 1; k >= 0; --k) {
      const int p = perm[k];
      if (p != k) {
        for (int i = tid; i < n; i += kBlock) {
          const double x = a[(size_t)i * n + k];
          a[(size_t)i * n + k] = a[(size_t)i * n + p];
          a[(size_t)i * n + p] = x;
        }
        __syncthreads();
      }
    }
    T* B = Wk.binv + boff;
    for (int q = tid; q < n * n; q += kBlock) B[q] = (T)a[q];
    if (Wk.binv64)   // mixed precision: the FP64 inverse too (fallback walkers run on it)
      for (int q = tid; q < n * n; q += kBlock) Wk.binv64[boff + q] = a[q];
  }
  if (tid == 0) {
    if (drift) drift[2 * w + sp] = Wk.logdet[2 * w + sp] - (singular ? NAN : logabs);
    Wk.logdet[2 * w + sp] = singular ? NAN : logabs;
    Wk.sign[2 * w + sp] = singular ? 0 : sgn;
    if (singular) atomicOr(Wk.status + w, 1 << sp);
  }
}

// ---------------------------------------------------------------------------
// The same elimination with the matrix held in registers (spin blocks up to
// kRegRebuildMax).  A G x G grid of threads (G = 16 for blocks up to 64, else
// 32) covers the matrix cyclically: thread (r0, c0), r0 = tid % G, c0 = tid / G,
// holds the entries (r0 + G i, c0 + G j), i, j < R, so a column's owners are G
// consecutive lanes (the pivot search is one reduction within them).  The small
// grid keeps a step's barriers to four waves for the common small blocks.  Rows are not swapped:
// step k takes as pivot the largest |a[i][k]| over the rows not yet used and
// records it, which is partial pivoting applied to the row-permuted matrix
// C = P A (C's row k = A's row p_k); the in-place elimination of C leaves
// C^-1[k][j] in physical row p_k, column j, and A^-1[k][p_j] = C^-1[k][j].
// Each entry sees the same operations, in the same order, as in k_rebuild, so
// both kernels give the same bits.  Per step only the pivot column and the
// pivot row pass through LDS (double-buffered by step parity: two barriers).
// ---------------------------------------------------------------------------
constexpr int kRegRebuildMax = 192;
constexpr int kRegBlock = 1024;

template <typename T, int R, int G>
__global__ __launch_bounds__(G * G) void k_rebuild_reg(SysParams P, Walkers<T> Wk, double* drift,
                                                           const uint32_t* sel, uint32_t sel_value) {
  __shared__ double scol[2][G * R];
  __shared__ double srow[2][G * R];
  __shared__ int spiv[G * R];    // physical row of each step's pivot
  __shared__ int sstep[G * R];   // step at which each physical row was the pivot
  __shared__ double spv[G * R];   // pivot of each step
  __shared__ double slog[G * R];
  __shared__ double sbest[2];
  __shared__ double samax[G * G / 64];
  const int w = blockIdx.x >> 1, sp = blockIdx.x & 1, tid = threadIdx.x;
  const int lane = tid & 63, wave = wave_of(tid);
  const int r0 = tid & (G - 1), c0 = tid / G;
  const int n = sp ? P.n_dn : P.n_up, off = sp ? P.n_up : 0;
  const int N = P.N;
  if (sel && sel[w] != sel_value) return;
  if (n == 0) {
    if (tid == 0) {
      if (drift) drift[2 * w + sp] = Wk.logdet[2 * w + sp];
      Wk.logdet[2 * w + sp] = 0.0;
      Wk.sign[2 * w + sp] = 1;
    }
    return;
  }
  for (int q = tid; q < 2 * G * R; q += (G * G)) {
    (&scol[0][0])[q] = 0.0;
    (&srow[0][0])[q] = 0.0;
  }
  double a[R][R];
  unsigned used = 0;   // bit i: row r0 + G i is padding or has been a pivot
  double amax = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int e = r0 + G * i;
    if (e < n) {
      const size_t item = (size_t)w * N + off + e;
      const size_t row = (size_t)(Wk.cur[item] ^ Wk.row_flip) * P.W * N + item;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int l = c0 + G * j;
        a[i][j] = l < n ? (Wk.val64 ? Wk.val64[row * P.S + l] : (double)Wk.vgl[row * kComp * P.S + l]) : 0.0;
        amax = fmax(amax, fabs(a[i][j]));
      }
    } else {
      used |= 1u << i;
#pragma unroll
      for (int j = 0; j < R; ++j) a[i][j] = 0.0;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
  if (lane == 0) samax[wave] = amax;
  __syncthreads();
  amax = samax[0];
  for (int q = 1; q < G * G / 64; ++q) amax = fmax(amax, samax[q]);
  // a pivot this small relative to the largest entry means a numerically singular matrix
  const double tiny = 1e-14 * amax;
  double logabs = 0.0;
  int sgn = 1;
  bool singular = false;
  for (int k = 0; k < n; ++k) {
    const int b = k & 1;
    const int jk = k / G;
    const bool colk = c0 == (k & (G - 1));   // this thread holds entries of column k
    double* sc = &scol[b][r0];           // scol[b][r0 + G i] = sc[G i]
    double* sr = &srow[b][c0];           // srow[b][c0 + G j] = sr[G j]
    if (colk) {
      // these G lanes own column k: publish it and find the pivot among the unused rows
      double best = -1.0;
      int bi = n;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (j != jk) continue;   // uniform: one register column is taken
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const double v = a[i][j];
          if (r0 + G * i < n) sc[G * i] = v;
          if (!((used >> i) & 1u) && fabs(v) > best) { best = fabs(v); bi = r0 + G * i; }
        }
      }
#pragma unroll
      for (int o = G / 2; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (r0 == 0) { spiv[k] = bi; sbest[b] = best; }
    }
    __syncthreads();
    const int p = uniform(spiv[k]);
    const double best = uniform(sbest[b]);
    if (!(best > tiny) || !isfinite(best)) { singular = true; break; }
    const int ip = p / G;
    const bool rowp = r0 == (p & (G - 1));   // this thread holds entries of the pivot row
    if (rowp) {
      used |= 1u << ip;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (i != ip) continue;   // uniform: one register row is taken
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (c0 + G * j < n) sr[G * j] = a[i][j];
      }
    }
    __syncthreads();
    const double piv = uniform(srow[b][k]);
    const double pinv = 1.0 / piv;
    if (tid == 0) spv[k] = piv;
    // scaled pivot row; the pivot column's entry becomes 1 / piv
    double rs[R];
#pragma unroll
    for (int j = 0; j < R; ++j) rs[j] = (j == jk && colk) ? pinv : sr[G * j] * pinv;
    // column k restarts from zero, so the update leaves -a[i][k] / piv there
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (j != jk) continue;
#pragma unroll
      for (int i = 0; i < R; ++i) a[i][j] = colk ? 0.0 : a[i][j];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const double f = sc[G * i];
#pragma unroll
      for (int j = 0; j < R; ++j) a[i][j] = a[i][j] - f * rs[j];
    }
    // the pivot row itself becomes the scaled row
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (i != ip) continue;
#pragma unroll
      for (int j = 0; j < R; ++j) a[i][j] = rowp ? rs[j] : a[i][j];
    }
  }
  if (!singular) {
    for (int k = tid; k < n; k += (G * G)) sstep[spiv[k]] = k;
    __syncthreads();
    const size_t boff = (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
    T* B = Wk.binv + boff;
    double* B64 = Wk.binv64 ? Wk.binv64 + boff : nullptr;   // mixed precision: the FP64 inverse too
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = r0 + G * i;
      if (e >= n) continue;
      const size_t orow = (size_t)sstep[e] * n;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int l = c0 + G * j;
        if (l < n) {
          B[orow + spiv[l]] = (T)a[i][j];
          if (B64) B64[orow + spiv[l]] = a[i][j];
        }
      }
    }
    for (int k = tid; k < n; k += (G * G)) slog[k] = log(fabs(spv[k]));
    __syncthreads();
    if (tid == 0) {
      for (int k = 0; k < n; ++k) {
        logabs += slog[k];
        if (spv[k] < 0.0) sgn = -sgn;
      }
      // sign of the permutation k -> p_k: (-1)^(n - number of cycles)
      int cycles = 0;
      for (int s0 = 0; s0 < n; ++s0) {
        if (sstep[s0] < 0) continue;
        ++cycles;
        for (int t = s0; sstep[t] >= 0;) {
          const int nx = spiv[t];
          sstep[t] = -1;
          t = nx;
        }
      }
      if ((n - cycles) & 1) sgn = -sgn;
    }
  }
  if (tid == 0) {
    if (drift) drift[2 * w + sp] = Wk.logdet[2 * w + sp] - (singular ? NAN : logabs);
    Wk.logdet[2 * w + sp] = singular ? NAN : logabs;
    Wk.sign[2 * w + sp] = singular ? 0 : sgn;
    if (singular) atomicOr(Wk.status + w, 1 << sp);
  }
}

// ---------------------------------------------------------------------------
// The same elimination, blocked, for spin blocks beyond kRegRebuildMax.  The
// matrix stays in the FP64 scratch buffer and its columns are taken in panels
// of PB.  A panel's PB steps run in LDS on the panel columns (pivot among the
// unused rows, scaling, elimination, as above); every other column then takes
// the panel's PB steps in one pass, so the matrix is read and written once per
// panel instead of once per step.  For a column c outside the panel, with
// col_s the panel's column s just before step s and p_t the pivot row of step t:
//   r_t = (a[p_t][c] - sum_{s<t} col_s[p_t] r_s) / piv_t   (scaled pivot row)
//   a[i][c] <- a[i][c] - sum_s col_s[i] r_s                 (rows not pivots here)
//   a[p_t][c] <- r_t - sum_{s>t} col_s[p_t] r_s             (the panel's pivot rows)
// Each entry sees the operations of the sequential elimination in the same
// order, so the result has the same bits.
// ---------------------------------------------------------------------------
struct PanelLayout {
  size_t pan, cols, pinv, prow, piv, pstep, used, total;
};

__host__ __device__ inline PanelLayout panel_layout(int n, int pb) {
  PanelLayout L;
  size_t o = 0;
  L.pan = o; o += sizeof(double) * (size_t)n * pb;    // panel columns, row-major [n][pb]
  L.cols = o; o += sizeof(double) * (size_t)pb * n;   // col_s, [pb][n]
  L.pinv = o; o += sizeof(double) * pb;
  L.prow = o; o += sizeof(double) * pb;
  L.piv = o; o += sizeof(int) * (size_t)n;            // pivot row of each step
  L.pstep = o; o += sizeof(int) * (size_t)n;          // step within the current panel, or -1
  L.used = o; o += (size_t)n;
  L.total = (o + 15) & ~(size_t)15;
  return L;
}

template <typename T, int PB>
__global__ __launch_bounds__(kBlock) void k_rebuild_panel(SysParams P, Walkers<T> Wk, double* scratch,
                                                          double* drift, const uint32_t* sel, uint32_t sel_value) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double rv[kWaves];
  __shared__ int ri[kWaves];
  const int w = blockIdx.x >> 1, sp = blockIdx.x & 1, tid = threadIdx.x;
  const int lane = tid & 63, wave = wave_of(tid);
  const int n = sp ? P.n_dn : P.n_up, off = sp ? P.n_up : 0;
  const int N = P.N;
  if (sel && sel[w] != sel_value) return;
  if (n == 0) {
    if (tid == 0) {
      if (drift) drift[2 * w + sp] = Wk.logdet[2 * w + sp];
      Wk.logdet[2 * w + sp] = 0.0;
      Wk.sign[2 * w + sp] = 1;
    }
    return;
  }
  const PanelLayout lay = panel_layout(n, PB);
  double* pan = reinterpret_cast<double*>(smem + lay.pan);
  double* cols = reinterpret_cast<double*>(smem + lay.cols);
  double* spinv = reinterpret_cast<double*>(smem + lay.pinv);
  double* prow = reinterpret_cast<double*>(smem + lay.prow);
  int* spiv = reinterpret_cast<int*>(smem + lay.piv);
  int* pstep = reinterpret_cast<int*>(smem + lay.pstep);
  uint8_t* used = smem + lay.used;
  const size_t boff = (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
  double* a = scratch + boff;
  double amax = 0.0;
  for (int q = tid; q < n * n; q += kBlock) {
    const int k = q / n, l = q - k * n;
    const size_t item = (size_t)w * N + off + k;
    const int cb = Wk.cur[item] ^ Wk.row_flip;
    a[q] = Wk.val64 ? Wk.val64[((size_t)cb * P.W * N + item) * P.S + l]
                    : (double)Wk.vgl[((size_t)cb * P.W * N + item) * kComp * P.S + l];
    amax = fmax(amax, fabs(a[q]));
  }
  for (int i = tid; i < n; i += kBlock) used[i] = 0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
  if (lane == 0) rv[wave] = amax;
  __syncthreads();
  amax = fmax(fmax(rv[0], rv[1]), fmax(rv[2], rv[3]));
  // a pivot this small relative to the largest entry means a numerically singular matrix
  const double tiny = 1e-14 * amax;
  __syncthreads();
  double logabs = 0.0;
  int sgn = 1;
  bool singular = false;
  for (int k0 = 0; k0 < n; k0 += PB) {
    const int bw = min(PB, n - k0);
    // (1) the panel's columns into LDS
    for (int q = tid; q < n * bw; q += kBlock) {
      const int i = q / bw, t = q - i * bw;
      pan[i * PB + t] = a[(size_t)i * n + k0 + t];
    }
    for (int i = tid; i < n; i += kBlock) pstep[i] = -1;
    __syncthreads();
    for (int t = 0; t < bw; ++t) {
      // pivot: largest |pan[i][t]| over the unused rows (smallest index on ties)
      double best = -1.0;
      int bi = n;
      for (int i = tid; i < n; i += kBlock) {
        const double v = fabs(pan[i * PB + t]);
        if (!used[i] && v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) { rv[wave] = best; ri[wave] = bi; }
      __syncthreads();
      best = rv[0];
      bi = ri[0];
      for (int q = 1; q < kWaves; ++q)
        if (rv[q] > best || (rv[q] == best && ri[q] < bi)) { best = rv[q]; bi = ri[q]; }
      if (!(best > tiny) || !isfinite(best)) { singular = true; break; }
      const int p = bi;
      const double piv = pan[p * PB + t];
      const double pinv = 1.0 / piv;
      if (tid == 0) {
        logabs += log(fabs(piv));
        if (piv < 0.0) sgn = -sgn;
      }
      for (int i = tid; i < n; i += kBlock) cols[t * n + i] = pan[i * PB + t];
      if (tid < bw) prow[tid] = (tid == t) ? pinv : pan[p * PB + tid] * pinv;
      __syncthreads();   // everyone has read the reductions, column t and the pivot row
      if (tid == 0) {
        spiv[k0 + t] = p;
        pstep[p] = t;
        used[p] = 1;
        spinv[t] = pinv;
      }
      for (int q = tid; q < n * bw; q += kBlock) {
        const int i = q / bw, tt = q - i * bw;
        pan[i * PB + tt] = (i == p) ? prow[tt] : ((tt == t) ? 0.0 : pan[i * PB + tt]) - cols[t * n + i] * prow[tt];
      }
      __syncthreads();
    }
    if (singular) break;
    // (2) the panel back, and its steps applied to every other column (one column per thread)
    for (int q = tid; q < n * bw; q += kBlock) {
      const int i = q / bw, t = q - i * bw;
      a[(size_t)i * n + k0 + t] = pan[i * PB + t];
    }
    for (int c = tid; c < n; c += kBlock) {
      if (c >= k0 && c < k0 + bw) continue;
      double r[PB];
#pragma unroll
      for (int t = 0; t < PB; ++t) {
        r[t] = 0.0;
        if (t < bw) {
          const int pt = spiv[k0 + t];
          double v = a[(size_t)pt * n + c];
#pragma unroll
          for (int s2 = 0; s2 < t; ++s2) v = v - cols[s2 * n + pt] * r[s2];
          r[t] = v * spinv[t];
        }
      }
      constexpr int kRows = 8;   // rows in flight
      for (int i0 = 0; i0 < n; i0 += kRows) {
        double v[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) v[u] = a[(size_t)min(i0 + u, n - 1) * n + c];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
          const int i = i0 + u;
          if (i >= n) break;
          const int ps = pstep[i];   // the same for every thread
          if (ps < 0) {
#pragma unroll
            for (int s2 = 0; s2 < PB; ++s2)
              if (s2 < bw) v[u] = v[u] - cols[s2 * n + i] * r[s2];
          } else {
            double x = 0.0;
#pragma unroll
            for (int t = 0; t < PB; ++t) x = (t == ps) ? r[t] : x;
#pragma unroll
            for (int s2 = 0; s2 < PB; ++s2)
              if (s2 > ps && s2 < bw) x = x - cols[s2 * n + i] * r[s2];
            v[u] = x;
          }
          a[(size_t)i * n + c] = v[u];
        }
      }
    }
    __syncthreads();   // the matrix is current before the next panel is read
  }
  int* sstep = pstep;   // reused: step at which each physical row was the pivot
  if (!singular) {
    for (int k = tid; k < n; k += kBlock) sstep[spiv[k]] = k;
    __syncthreads();
    T* B = Wk.binv + boff;
    double* B64 = Wk.binv64 ? Wk.binv64 + boff : nullptr;   // mixed precision: the FP64 inverse too
    for (int q = tid; q < n * n; q += kBlock) {
      const int r = q / n, c = q - r * n;
      B[(size_t)sstep[r] * n + spiv[c]] = (T)a[q];
      if (B64) B64[(size_t)sstep[r] * n + spiv[c]] = a[q];
    }
    __syncthreads();
    if (tid == 0) {
      // sign of the permutation k -> p_k: (-1)^(n - number of cycles)
      int cycles = 0;
      for (int s0 = 0; s0 < n; ++s0) {
        if (sstep[s0] < 0) continue;
        ++cycles;
        for (int t = s0; sstep[t] >= 0;) {
          const int nx = spiv[t];
          sstep[t] = -1;
          t = nx;
        }
      }
      if ((n - cycles) & 1) sgn = -sgn;
    }
  }
  if (tid == 0) {
    if (drift) drift[2 * w + sp] = Wk.logdet[2 * w + sp] - (singular ? NAN : logabs);
    Wk.logdet[2 * w + sp] = singular ? NAN : logabs;
    Wk.sign[2 * w + sp] = singular ? 0 : sgn;
    if (singular) atomicOr(Wk.status + w, 1 << sp);
  }
}

template <typename T, int PB>
static hipError_t launch_rebuild_panel(const SysParams& P, const Walkers<T>& Wk, double* scratch, double* drift,
                                       hipStream_t st, const uint32_t* sel, uint32_t sel_value, size_t bytes) {
  if (bytes > 65536) {
    const hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_rebuild_panel<T, PB>));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_rebuild_panel<T, PB>), dim3(2 * P.W), dim3(kBlock), bytes, st, P, Wk, scratch, drift,
                     sel, sel_value);
  return hipGetLastError();
}

static int lds_budget_rebuild() {
  static int budget = -1;
  if (budget < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      budget = v;
    else
      budget = 65536;
  }
  return budget;
}

// ---------------------------------------------------------------------------
// FP64 refinement of the FP32 inverses before a measurement (mixed precision).
//
// Between full rebuilds the FP32 rank-one and delayed updates let B drift from
// A^-1 by a few FP32 units times the conditioning of A; the kinetic energy sums
// B[l][k] times orbital Laplacians with heavy cancellation, so that drift can
// reach 1e-4 of the energy.  One correction step X = B + B (I - A B), with the
// FP64 Slater matrix A, squares the relative error of the inverse.  The residual
// E = I - A B cancels to ~1e-6 and is formed on the FP64 matrix cores; the
// correction B E is that small relative to B, so it is formed on the FP32
// matrix cores from E rounded to FP32 (its rounding is far below that of the
// FP32 X).  Both products run in 64 x 64 output tiles staged through LDS; E
// goes to the scratch buffer, X to the buffer the measurement reads (binv
// itself is not changed, so a measurement never alters the chain).
// ---------------------------------------------------------------------------
// (16-wide k chunks: the staged panels take few registers, and the refinement runs four
// workgroups per compute unit)
constexpr int kTile = 64, kChunk = 16;
constexpr int kLs = kChunk + 1;    // padded LDS row strides (fewer bank conflicts)
constexpr int kRs = kTile + 2;
constexpr int kPerThread = kTile * kChunk / kBlock;   // panel entries each thread stages

// C[i][k] = sum_l Lf(i, l) Rf(l, k) for i, k < n; epi(i, k, C[i][k]) stores each
// result.  All threads of the block call it; each wave owns a 32 x 32 quadrant of a
// 64 x 64 output tile.  The panels of the next k-chunk are loaded into registers while
// the matrix cores work on the current chunk from LDS.
template <typename V, typename LF, typename RF, typename EF>
__device__ __forceinline__ void gemm_tiles(int n, LF Lf, RF Rf, EF epi, V* sL, V* sR) {
  typedef Mfma<V> M;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_of(tid);
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int nt = (n + kTile - 1) / kTile;
  const int nc = (n + kChunk - 1) / kChunk;
  for (int t = 0; t < nt * nt; ++t) {
    const int i0 = (t / nt) * kTile, k0 = (t % nt) * kTile;
    typename M::v4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = typename M::v4{V(0), V(0), V(0), V(0)};
    V rl[kPerThread], rr[kPerThread];
    auto fetch = [&](int l0) {
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) {
        const int q = tid + e * kBlock;
        const int r = q / kChunk, c = q % kChunk;          // left panel: row r, column c
        // unconditional loads from clamped indices, out-of-range entries zeroed
        const int i = i0 + r, l = l0 + c;
        const V vl = Lf(i < n ? i : n - 1, l < n ? l : n - 1);
        rl[e] = (i < n && l < n) ? vl : V(0);
        const int rr2 = q / kTile, cc = q % kTile;         // right panel: row rr2, column cc
        const int l2 = l0 + rr2, k = k0 + cc;
        const V vr = Rf(l2 < n ? l2 : n - 1, k < n ? k : n - 1);
        rr[e] = (l2 < n && k < n) ? vr : V(0);
      }
    };
    fetch(0);
    for (int ch = 0; ch < nc; ++ch) {
#pragma unroll
      for (int e = 0; e < kPerThread; ++e) {
        const int q = tid + e * kBlock;
        sL[(q / kChunk) * kLs + q % kChunk] = rl[e];
        sR[(q / kTile) * kRs + q % kTile] = rr[e];
      }
      __syncthreads();
      if (ch + 1 < nc) fetch((ch + 1) * kChunk);   // in flight during the products below
#pragma unroll
      for (int kk = 0; kk < kChunk; kk += 4) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const V av = sL[(wr + 16 * a + li) * kLs + kk + lk];
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const V bv = sR[(kk + lk) * kRs + wc + 16 * b + li];
            acc[a][b] = M::mma(av, bv, acc[a][b]);
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + wr + 16 * a + M::row(lane, r), k = k0 + wc + 16 * b + li;
          if (i < n && k < n) epi(i, k, acc[a][b][r]);
        }
  }
}

// The FP64 product.
template <typename LF, typename RF, typename EF>
__device__ __forceinline__ void gemm64(int n, LF Lf, RF Rf, EF epi, double* sL, double* sR) {
  gemm_tiles<double>(n, Lf, Rf, epi, sL, sR);
}

// Sum over the workgroup (every thread gets it; fixed order).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum_dpp(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) t += red[q];
  return t;
}

template <typename T>
__device__ __forceinline__ void refine_spin(const SysParams& P, const Walkers<T>& Wk, double* scratch, int w,
                                            int sp) {
  __shared__ double sL[kTile * kLs];
  __shared__ double sR[kChunk * kRs];
  __shared__ size_t arow[kMaxSpin];   // row offsets in val64 (not pointers: the loads stay global, not flat)
  __shared__ double red[kWaves];
  const int n = sp ? P.n_dn : P.n_up, off = sp ? P.n_up : 0;
  if (Wk.fb && Wk.fb[w]) return;   // an FP64 fallback walker is measured on its FP64 inverse
  if (sp == 0 && threadIdx.x == 0 && Wk.eta_age) Wk.eta_age[w] = 0u;
  if (n == 0) {
    if (threadIdx.x == 0 && Wk.eta) Wk.eta[4 * w + sp] = Wk.eta[4 * w + 2 + sp] = 0.0;
    return;
  }
  const int N = P.N;
  const size_t boff = (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
  const T* B = Wk.binv + boff;
  T* X = Wk.xinv + boff;
  float* E = reinterpret_cast<float*>(scratch + boff);
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const size_t item = (size_t)w * N + off + i;
    arow[i] = ((size_t)Wk.cur[item] * P.W * N + item) * P.S;
  }
  __syncthreads();
  // E = I - A B in FP64 (A B is the identity up to ~1e-6: the difference needs FP64 products);
  // E itself is small and is kept in FP32
  double e2 = 0.0, x2 = 0.0;   // ||E||_F^2 and ||X||_F^2 partials (the guard band's inverse error)
  gemm64(n, [&](int i, int l) { return Wk.val64[arow[i] + l]; },
         [&](int l, int k) { return (double)B[(size_t)l * n + k]; },
         [&](int i, int k, double c) {
           const double e = (i == k ? 1.0 : 0.0) - c;
           e2 += e * e;
           E[(size_t)i * n + k] = (float)e;
         }, sL, sR);
  __syncthreads();   // E (global) complete before it is read
  if (Wk.ecol)   // each column's residual norm, for the guard band of the next sweep's ratios
    for (int k = threadIdx.x; k < n; k += kBlock) {
      double c2 = 0.0;
#pragma unroll 8
      for (int i = 0; i < n; ++i) {   // (unrolled: eight loads in flight, the sum still in order)
        const double e = (double)E[(size_t)i * n + k];
        c2 += e * e;
      }
      Wk.ecol[(size_t)w * N + off + k] = (float)sqrt(c2);
    }
  // X = B + B E: the correction B E is ~1e-6 of B, so FP32 products (relative error ~1e-5 of
  // the correction, ~1e-11 of X) are far inside the FP32 rounding of the stored X
  gemm_tiles<float>(n, [&](int i, int l) { return (float)B[(size_t)i * n + l]; },
                    [&](int l, int k) { return E[(size_t)l * n + k]; },
                    [&](int i, int k, float c) {
                      const T x = (T)((double)B[(size_t)i * n + k] + (double)c);
                      x2 += (double)x * (double)x;
                      X[(size_t)i * n + k] = x;
                    },
                    reinterpret_cast<float*>(sL), reinterpret_cast<float*>(sR));
  e2 = block_sum(e2, red);   // (its barriers also complete X before the copy below)
  x2 = block_sum(x2, red);
  if (threadIdx.x == 0 && Wk.eta) {
    Wk.eta[4 * w + sp] = sqrt(e2);
    Wk.eta[4 * w + 2 + sp] = sqrt(x2);
  }
  // The chain goes on from the refined inverse: with A B = I - E, A X = I - E^2, so the FP32
  // updates' drift is squared away at every measurement instead of accumulating until the next
  // full rebuild (the decisions, taken to FP64 accuracy by the guard, do not change).
  if (Wk.fb) {
    T* Bw = Wk.binv + boff;
    for (int q = threadIdx.x; q < n * n; q += kBlock) Bw[q] = X[q];
  }
}

// sel (nullable): only the walkers with sel[w] == sel_value are refined.
template <typename T>
__global__ __launch_bounds__(kBlock, 4) void k_refine(SysParams P, Walkers<T> Wk, double* scratch,
                                                   const uint32_t* sel, uint32_t sel_value) {
  if (sel && sel[blockIdx.x >> 1] != sel_value) return;
  refine_spin<T>(P, Wk, scratch, blockIdx.x >> 1, blockIdx.x & 1);
}

// Batched: block b refines spin b & 1 of (system, walker) fmap[b >> 1].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_refine_batched(const SysDev<T>* __restrict__ sd,
                                                           const int2* __restrict__ fmap) {
  __shared__ SysDev<T> s;
  const int2 m = fmap[blockIdx.x >> 1];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(sd + m.x);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&s);
    for (int q = threadIdx.x; q < (int)(sizeof(SysDev<T>) / 4); q += kBlock) dst[q] = src[q];
  }
  __syncthreads();
  refine_spin<T>(s.P, s.W, s.scratch, m.y, blockIdx.x & 1);
}

template <typename T>
hipError_t launch_refine(const SysParams& P, const Walkers<T>& Wk, double* scratch, hipStream_t st,
                         const uint32_t* sel, uint32_t sel_value) {
  if (P.n_up > kMaxSpin || P.n_dn > kMaxSpin || !Wk.val64 || !Wk.xinv) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_refine<T>, dim3(2 * P.W), dim3(kBlock), 0, st, P, Wk, scratch, sel, sel_value);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_refine_batched(const SysDev<T>* sd, const int2* fmap, int n_walkers, hipStream_t st) {
  if (n_walkers <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_batched<T>, dim3(2 * n_walkers), dim3(kBlock), 0, st, sd, fmap);
  return hipGetLastError();
}

template hipError_t launch_refine<float>(const SysParams&, const Walkers<float>&, double*, hipStream_t,
                                         const uint32_t*, uint32_t);

// ---------------------------------------------------------------------------
// FP64 fallback of ill-conditioned walkers (mixed precision).
//
// A walker's FP32 inverse B can carry the FP64 chain's decisions only while its
// error is small: with A B = I - E the ratio of a proposal v errs by at most
// ||v^T B|| ||E||_F.  An inverse rounded to FP32 has ||E|| of the order of the
// condition number of A times 2^-24, so an ill-conditioned walker (two electrons
// of one spin close together at a uniform start, for instance) cannot be run in
// FP32 at all.  After every full rebuild and every measurement the walkers are
// checked: a measured ||E||_F above kEtaRebuild (drift of the FP32 updates) has
// the walker's inverse rebuilt in FP64; a fresh FP32 rounding of the FP64 inverse
// whose residual still exceeds kEtaEnter sends the walker to the FP64 fallback
// (its chain runs in FP64 on binv64, its kinetic energy reads binv64), and a
// fallback walker whose FP32 rounding falls below kEtaLeave returns to FP32.
//
// mark[w]: 1 = rebuild and check, 2 = check a fallback walker, 3 = refine (back in
// FP32 after a check), 0 = nothing.
// ---------------------------------------------------------------------------

// mark[w] after a measurement's refinement (all = 1: after a full rebuild of every walker).
__global__ __launch_bounds__(kBlock) void k_fb_mark(int W, const double* __restrict__ eta, const int* __restrict__ fb,
                                                    uint32_t* __restrict__ mark, int all) {
  const int w = blockIdx.x * kBlock + threadIdx.x;
  if (w >= W) return;
  mark[w] = all ? 1u : (fb[w] ? 2u : (fmax(eta[4 * w], eta[4 * w + 1]) > kEtaRebuild ? 1u : 0u));
}

hipError_t launch_fb_mark(int W, const double* eta, const int* fb, uint32_t* mark, int all, hipStream_t st) {
  hipLaunchKernelGGL(k_fb_mark, dim3((W + kBlock - 1) / kBlock), dim3(kBlock), 0, st, W, eta, fb, mark, all);
  return hipGetLastError();
}

// eta[w] = ||I - A fl32(B64)||_F and ||B64||_F per spin for the walkers with mark 1 or 2: the
// error an FP32 copy of the FP64 inverse would start from (FP64 products, A = the FP64 rows).
__global__ __launch_bounds__(kBlock) void k_fb_residual(SysParams P, Walkers<float> Wk, double* scratch,
                                                        const uint32_t* mark) {
  __shared__ double sL[kTile * kLs];
  __shared__ double sR[kChunk * kRs];
  __shared__ size_t arow[kMaxSpin];   // row offsets in val64 (not pointers: the loads stay global, not flat)
  __shared__ double red[kWaves];
  const int w = blockIdx.x >> 1, sp = blockIdx.x & 1, tid = threadIdx.x;
  if (mark[w] != 1u && mark[w] != 2u) return;
  if (sp == 0 && tid == 0) Wk.eta_age[w] = 0u;
  const int n = sp ? P.n_dn : P.n_up, off = sp ? P.n_up : 0;
  if (n == 0) {
    if (tid == 0) Wk.eta[4 * w + sp] = Wk.eta[4 * w + 2 + sp] = 0.0;
    return;
  }
  const int N = P.N;
  const size_t boff = (size_t)w * P.bstride + (sp ? (size_t)P.n_up * P.n_up : 0);
  const double* B = Wk.binv64 + boff;
  float* E = reinterpret_cast<float*>(scratch + boff);
  for (int i = tid; i < n; i += kBlock) {
    const size_t item = (size_t)w * N + off + i;
    arow[i] = ((size_t)Wk.cur[item] * P.W * N + item) * P.S;
  }
  __syncthreads();
  double e2 = 0.0, b2 = 0.0;
  gemm64(n, [&](int i, int l) { return Wk.val64[arow[i] + l]; },
         [&](int l, int k) { return (double)(float)B[(size_t)l * n + k]; },
         [&](int i, int k, double c) {
           const double e = (i == k ? 1.0 : 0.0) - c;
           e2 += e * e;
           E[(size_t)i * n + k] = (float)e;
         }, sL, sR);
  __syncthreads();   // E complete before its columns are read
  // each column's residual norm: the guard band of the next sweep's ratios for a walker that goes
  // on from this FP32 copy (the same numbers a refinement of it would record)
  for (int k = tid; k < n; k += kBlock) {
    double c2 = 0.0;
#pragma unroll 8
    for (int i = 0; i < n; ++i) {   // (unrolled: eight loads in flight, the sum still in order)
      const double e = (double)E[(size_t)i * n + k];
      c2 += e * e;
    }
    Wk.ecol[(size_t)w * N + off + k] = (float)sqrt(c2);
  }
  for (int q = tid; q < n * n; q += kBlock) b2 += B[q] * B[q];
  e2 = block_sum(e2, red);
  b2 = block_sum(b2, red);
  if (tid == 0) {
    Wk.eta[4 * w + sp] = sqrt(e2);
    Wk.eta[4 * w + 2 + sp] = sqrt(b2);
  }
}

hipError_t launch_fb_residual(const SysParams& P, const Walkers<float>& Wk, double* scratch, const uint32_t* mark,
                              hipStream_t st) {
  if (P.n_up > kMaxSpin || P.n_dn > kMaxSpin || !Wk.binv64 || !Wk.eta || !Wk.ecol) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fb_residual, dim3(2 * P.W), dim3(kBlock), 0, st, P, Wk, scratch, mark);
  return hipGetLastError();
}

// The decision for the checked walkers: FP64 fallback while the FP32 rounding's residual
// exceeds kEtaEnter (kEtaLeave for a walker already in fallback).  A walker returning to
// FP32 takes binv = fl32(binv64) and mark 3 (its refinement is due); mark 1 counts an early
// rebuild when early != 0.
__global__ __launch_bounds__(kBlock) void k_fb_decide(SysParams P, Walkers<float> Wk, uint32_t* mark, int early) {
  const int w = blockIdx.x, tid = threadIdx.x;
  const uint32_t m = mark[w];
  if (m != 1u && m != 2u) return;
  const int was = Wk.fb[w];
  const double eta = fmax(Wk.eta[4 * w], Wk.eta[4 * w + 1]);
  const int now = eta > (was ? kEtaLeave : kEtaEnter) ? 1 : 0;
  if (!now && m == 2u) {
    const size_t off = (size_t)w * P.bstride;
    for (int q = tid; q < P.bstride; q += kBlock) Wk.binv[off + q] = (float)Wk.binv64[off + q];
  }
  __syncthreads();
  if (tid == 0) {
    Wk.fb[w] = now;
    mark[w] = now ? 0u : 3u;
    if (early && m == 1u) Wk.pstat[2 * w] += 1u;
  }
}

hipError_t launch_fb_decide(const SysParams& P, const Walkers<float>& Wk, uint32_t* mark, int early, hipStream_t st) {
  hipLaunchKernelGGL(k_fb_decide, dim3(P.W), dim3(kBlock), 0, st, P, Wk, mark, early);
  return hipGetLastError();
}

// A walker back in FP32 after a check (mark 3) goes on from binv = fl32(B64), a fresh rounding of
// an FP64 inverse, which a refinement (itself stored in FP32) would not improve: the measurement
// reads that copy, and k_fb_residual has recorded its residuals.
__global__ __launch_bounds__(kBlock) void k_fb_adopt(SysParams P, Walkers<float> Wk, const uint32_t* mark) {
  const int w = blockIdx.x;
  if (mark[w] != 3u) return;
  const size_t off = (size_t)w * P.bstride;
  const int nb = P.n_up * P.n_up + P.n_dn * P.n_dn;
  for (int q = threadIdx.x; q < nb; q += kBlock) Wk.xinv[off + q] = Wk.binv[off + q];
}

hipError_t launch_fb_adopt(const SysParams& P, const Walkers<float>& Wk, const uint32_t* mark, hipStream_t st) {
  if (!Wk.xinv) return hipSuccess;
  hipLaunchKernelGGL(k_fb_adopt, dim3(P.W), dim3(kBlock), 0, st, P, Wk, mark);
  return hipGetLastError();
}

template hipError_t launch_refine_batched<float>(const SysDev<float>*, const int2*, int, hipStream_t);

template <typename T>
hipError_t launch_rebuild(const SysParams& P, const Walkers<T>& Wk, double* scratch, double* drift,
                          hipStream_t st, const uint32_t* sel, uint32_t sel_value, bool beside_other) {
  if (P.n_up > kMaxSpin || P.n_dn > kMaxSpin) return hipErrorInvalidValue;
  const int nmax = P.n_up > P.n_dn ? P.n_up : P.n_dn;
  // QMC_REBUILD_GLOBAL=1 takes the global-memory elimination for every size (lets the
  // tests compare the two kernels)
  const char* fg = getenv("QMC_REBUILD_GLOBAL");
  // A selective rebuild (a few walkers) beside a kernel that fills the device takes the panel
  // kernel for blocks beyond 64 when it fits: its 256-thread workgroups are placed beside the
  // other kernel's workgroups, where a 1024-thread one waits for a whole compute unit to drain
  // (measured at 384 electrons: 2.0 against 3.5 ms per launch beside the gather; alone the
  // register elimination of one walker takes 0.4 ms and the panel one 2.6 ms).
  const bool beside = beside_other && sel && nmax > 64;
  if (!(fg && fg[0] == '1') && nmax <= kRegRebuildMax &&
      !(beside && panel_layout(nmax, 16).total <= (size_t)lds_budget_rebuild())) {
    const dim3 grid(2 * P.W);
    if (nmax <= 64) {
      const dim3 block(16 * 16);
      switch ((nmax + 15) / 16) {
        case 1: hipLaunchKernelGGL((k_rebuild_reg<T, 1, 16>), grid, block, 0, st, P, Wk, drift, sel, sel_value); break;
        case 2: hipLaunchKernelGGL((k_rebuild_reg<T, 2, 16>), grid, block, 0, st, P, Wk, drift, sel, sel_value); break;
        case 3: hipLaunchKernelGGL((k_rebuild_reg<T, 3, 16>), grid, block, 0, st, P, Wk, drift, sel, sel_value); break;
        default: hipLaunchKernelGGL((k_rebuild_reg<T, 4, 16>), grid, block, 0, st, P, Wk, drift, sel, sel_value); break;
      }
      return hipGetLastError();
    }
    const dim3 block(kRegBlock);
    switch ((nmax + 31) / 32) {
      case 3: hipLaunchKernelGGL((k_rebuild_reg<T, 3, 32>), grid, block, 0, st, P, Wk, drift, sel, sel_value); break;
      case 4: hipLaunchKernelGGL((k_rebuild_reg<T, 4, 32>), grid, block, 0, st, P, Wk, drift, sel, sel_value); break;
      case 5: hipLaunchKernelGGL((k_rebuild_reg<T, 5, 32>), grid, block, 0, st, P, Wk, drift, sel, sel_value); break;
      default: hipLaunchKernelGGL((k_rebuild_reg<T, 6, 32>), grid, block, 0, st, P, Wk, drift, sel, sel_value); break;
    }
    return hipGetLastError();
  }
  if (!(fg && fg[0] == '1')) {
    const size_t b16 = panel_layout(nmax, 16).total, b8 = panel_layout(nmax, 8).total;
    const size_t budget = (size_t)lds_budget_rebuild();
    if (b16 <= budget) return launch_rebuild_panel<T, 16>(P, Wk, scratch, drift, st, sel, sel_value, b16);
    if (b8 <= budget) return launch_rebuild_panel<T, 8>(P, Wk, scratch, drift, st, sel, sel_value, b8);
  }
  hipLaunchKernelGGL(k_rebuild<T>, dim3(2 * P.W), dim3(kBlock), 0, st, P, Wk, scratch, drift, sel, sel_value);
  return hipGetLastError();
}

template hipError_t launch_rebuild<double>(const SysParams&, const Walkers<double>&, double*, double*,
                                           hipStream_t, const uint32_t*, uint32_t, bool);
template hipError_t launch_rebuild<float>(const SysParams&, const Walkers<float>&, double*, double*,
                                          hipStream_t, const uint32_t*, uint32_t, bool);

hipError_t linalg_lds_limits() {
  const void* ks[] = {reinterpret_cast<const void*>(&k_rebuild_panel<double, 16>),
                      reinterpret_cast<const void*>(&k_rebuild_panel<double, 8>),
                      reinterpret_cast<const void*>(&k_rebuild_panel<float, 16>),
                      reinterpret_cast<const void*>(&k_rebuild_panel<float, 8>)};
  for (const void* k : ks) {
    const hipError_t e = allow_dynamic_lds(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qmc
