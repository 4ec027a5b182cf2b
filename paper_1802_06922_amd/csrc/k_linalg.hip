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
                                                    double* drift) {
  __shared__ double scol[kMaxSpin];
  __shared__ int perm[kMaxSpin];
  __shared__ double rv[kWaves];
  __shared__ int ri[kWaves];
  const int w = blockIdx.x >> 1, sp = blockIdx.x & 1, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int n = sp ? P.n_dn : P.n_up, off = sp ? P.n_up : 0;
  const int N = P.N;
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
    const int cb = Wk.cur[item];
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
  }
  if (tid == 0) {
    if (drift) drift[2 * w + sp] = Wk.logdet[2 * w + sp] - (singular ? NAN : logabs);
    Wk.logdet[2 * w + sp] = singular ? NAN : logabs;
    Wk.sign[2 * w + sp] = singular ? 0 : sgn;
    if (singular) atomicOr(Wk.status + w, 1 << sp);
  }
}

template <typename T>
hipError_t launch_rebuild(const SysParams& P, const Walkers<T>& Wk, double* scratch, double* drift,
                          hipStream_t st) {
  if (P.n_up > kMaxSpin || P.n_dn > kMaxSpin) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rebuild<T>, dim3(2 * P.W), dim3(kBlock), 0, st, P, Wk, scratch, drift);
  return hipGetLastError();
}

template hipError_t launch_rebuild<double>(const SysParams&, const Walkers<double>&, double*, double*,
                                           hipStream_t);
template hipError_t launch_rebuild<float>(const SysParams&, const Walkers<float>&, double*, double*,
                                          hipStream_t);

}  // namespace qmc
